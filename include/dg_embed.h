/*
 * dg_embed.h - C ABI of a small DGSEM solver that embeds the sliding-mesh mortar operator
 * (mortar.h) in a whole discretization, to check that the operator keeps the scheme's
 * order of accuracy (Duerrwaechter et al., arXiv 2008.04356, Sec. 5.2: a periodic
 * Cartesian box whose central slab slides, errors of order N + 1).
 *
 * The solver: compressible Euler or Navier-Stokes equations in conservative variables on
 * the periodic box [0, L]^3 with K x K x K hexahedral elements of edge h = L / K, the DGSEM of
 * Sec. 3 (Legendre-Gauss nodes, tensor-product Lagrange basis, weak form with the exact
 * diagonal mass matrix of Gauss collocation, Lax-Friedrichs surface fluxes; for
 * Navier-Stokes the gradients of the first Bassi-Rebay method: lifted with the face
 * average of the states, viscous face fluxes the average of both sides').  The
 * element layers j_lo <= j < j_hi along x2 form the moving slab: it translates along x1
 * with the constant grid velocity vg (its elements' nodes sit at x + vg t), and in it
 * the flux is the ALE flux F - vg U e1 (Sec. 2).  The two planes x2 = j_lo h and
 * x2 = j_hi h are sliding interfaces: their fluxes come from the mortar operator,
 * called by the driver between dg_prolong_interfaces and dg_rhs.
 *
 * Layouts (device arrays, double):
 *   U, dU, R   [n_elem][5][NP^3], element e = i + K (j + K k) (i along x1, j along x2,
 *              k along x3), node a + NP (b + NP c) (a along x1, b along x2, c along x3);
 *   FF         [3][n_elem][5][NP^2]: flux in the +e_d direction through the + face of
 *              element e in direction d, face point (b + NP c), (a + NP c), (a + NP b)
 *              for d = 0, 1, 2;
 *   interface  arrays of the mortar operator, [5][NP^2][K^2]: face (i, k) is column
 *              i + K k, point a + NP c (p_par along x1, p_perp along x3).  Interface 0
 *              is the plane x2 = j_lo h, interface 1 the plane x2 = j_hi h; for both the
 *              operator's static side is the element layer below the plane (normal +e2),
 *              its moving side the layer above.
 * Every call is asynchronous on stream and allocates nothing; 0 on success, -1 for an
 * invalid argument, -4 for a HIP error.
 */
#ifndef DG_EMBED_H
#define DG_EMBED_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dg_grid {
    int32_t N;          /* polynomial degree, 1 <= N <= 7 */
    int32_t K;          /* elements per direction */
    int32_t j_lo, j_hi; /* moving slab: element layers j_lo <= j < j_hi (0 < j_lo < j_hi < K) */
    double L;           /* box edge */
    double vg;          /* grid velocity of the slab along x1 */
    double gamma;       /* ratio of specific heats */
    double rho0, amp, u0, p0;  /* exact solution (dg_exact_state) */
    const double *basis; /* device: the tables written by dg_basis_tables */
    double mu, Pr;      /* viscosity and Prandtl number: mu > 0 selects Navier-Stokes */
} dg_grid;

/* Bytes of the device table buffer dg_basis_tables fills for degree N. */
int64_t dg_basis_bytes(int N);

/* Host-side tables of degree N into host buffer tab (dg_basis_bytes(N) bytes): Gauss
 * nodes and weights, l_j(-1), l_j(+1) and the weak-form derivative matrix
 * Dw[i][m] = (w_m / w_i) l_i'(x_m).  The caller copies them to the device and passes the
 * device copy as grid->basis. */
int dg_basis_tables(int N, double *tab);

/* The exact solution used here: a density wave carried by a uniform flow,
 *   rho = rho0 + amp sin(2 pi (x1 + x2 + x3 - 3 u0 t) / L), velocity (u0, u0, u0), p = p0,
 * an exact solution of the Euler equations; for Navier-Stokes the heat flux of its
 * temperature field needs the energy source -k/R p0 laplacian(1/rho), which dg_rhs adds.
 * Writes the conservative state of every node at time t into U. */
int dg_exact_state(const dg_grid *g, double t, double *U, void *stream);

/* Navier-Stokes, first Bassi-Rebay lifting: the average of both sides' states on every
 * conforming face into UF ([3][n_elem][5][NP^2], layout of FF). */
int dg_face_states(const dg_grid *g, const double *U, double *UF, void *stream);

/* The lifted gradients Q ([n_elem][3][5][NP^3]: dU_v/dx_d per node) from the states, the
 * conforming faces' averages UF and the two sliding planes' lifting terms of the mortar
 * operator (mortar_lifting outputs Ls[i], Lm[i], [3][5][NP^2][K^2], normal +e2, dS = 1). */
int dg_gradients(const dg_grid *g, const double *U, const double *UF, const double *Ls0,
                 const double *Lm0, const double *Ls1, const double *Lm1, double *Q, void *stream);

/* The two interfaces' face gradients for the mortar operator: Gs[i], Gm[i]
 * ([3][5][NP^2][K^2]). */
int dg_prolong_interface_gradients(const dg_grid *g, const double *Q, double *Gs0, double *Gm0,
                                   double *Gs1, double *Gm1, void *stream);

/* Face fluxes of all conforming faces (the sliding-interface faces are left to the mortar
 * operator) into FF; Q = NULL for Euler, else the lifted gradients (viscous fluxes). */
int dg_face_fluxes(const dg_grid *g, const double *U, const double *Q, double *FF, void *stream);

/* The two interfaces' face states for the mortar operator: Us[i], Um[i] ([5][NP^2][K^2])
 * of interface i = 0, 1 (static = the layer below, moving = the layer above). */
int dg_prolong_interfaces(const dg_grid *g, const double *U, double *Us0, double *Um0,
                          double *Us1, double *Um1, void *stream);

/* Right-hand side dU = volume + surface terms (+ the manufactured source at time t for
 * Navier-Stokes); Q = NULL for Euler.  The surface terms of the interface faces are the
 * mortar operator's outputs Fs[i] (static side, the + face of the layer below) and Fm[i]
 * (moving side, the - face of the layer above), both in the +e2 direction. */
int dg_rhs(const dg_grid *g, const double *U, const double *Q, const double *FF,
           const double *Fs0, const double *Fm0, const double *Fs1, const double *Fm1, double t,
           double *dU, void *stream);

/* One stage of a low-storage Runge-Kutta scheme: R = a R + dt dU; U = U + b R
 * (n values each). */
int dg_rk_stage(double *U, double *R, const double *dU, double a, double b, double dt,
                int64_t n, void *stream);

/* Per element, the Gauss-quadrature integral of (rho_h - rho_exact)^2 at time t into
 * err[n_elem] (the L2 error is the square root of their sum). */
int dg_density_error(const dg_grid *g, const double *U, double t, double *err, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* DG_EMBED_H */
