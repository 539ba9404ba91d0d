/*
 * mortar.h - C ABI of the MI355X sliding-mesh mortar interface operator.
 *
 * The operator is the per-Runge-Kutta-stage coupling of a static and a moving
 * sub-domain across a sliding interface in a DGSEM compressible Navier-Stokes
 * solver (Duerrwaechter et al., "An Efficient Sliding Mesh Interface Method for
 * High-Order Discontinuous Galerkin Schemes", arXiv 2008.04356):
 *   1. the displacement Delta = (n + s) l_par gives the sub-face fraction s and the
 *      static-to-moving face pairing (Sec. 4.3, index relation);
 *   2. the 1D L2 projection matrices of the Lagrange basis onto the two mortar
 *      sub-intervals are rebuilt for s (Sec. 3.2, Eqs. for M, S and P);
 *   3. both sides' face states (and lifted gradients) are projected onto the mortars,
 *      the Riemann (Roe with Harten-Hyman fix, or Lax-Friedrichs) plus BR1 viscous flux
 *      is evaluated once per mortar point, and the flux is projected back onto the
 *      static and the moving faces (Sec. 3.3, five-step procedure; Sec. 4.2);
 *   4. when the displacement crosses a whole face, the sorted mortar index array A and
 *      its inverse map m are rebuilt (Sec. 4.4, Appendix A).
 *
 * Data layout (every array, host or device):
 *   N = polynomial degree, NP = N + 1, P = NP * NP points per face, point
 *   p = p_par + NP * p_perp in interface-aligned orientation (p_par ascending along the
 *   sliding direction on both sides, p_perp ascending across it);
 *   states    U[5][P][n_face]      conservative (rho, rho u, rho v, rho w, rho E);
 *   gradients G[3][5][P][n_face]   G[d][v] = d U_v / d x_d (BR1 lifted, NS only);
 *   fluxes    F[5][P][n_face]      surface flux times surface element, in the STATIC
 *                                  side's normal direction on both sides (the caller's
 *                                  surface integral applies the sign of each side);
 *   metrics   M[4][P][n_face_s]    static-side (n_x, n_y, n_z, dS) per point; both are
 *                                  interpolated to the mortar nodes and the normal is
 *                                  scaled to unit length there (on curved interfaces the
 *                                  interpolant of unit normals is shorter between nodes).
 *   The face (i_par, i_perp) of a side is column face_id[i_perp * n_par + i_par].
 *   Performance: the rows of an array are n_face elements apart; when that stride is a
 *   multiple of a large power of two, the rows of all (variable, point) planes fall into
 *   the same cache sets and lines are fetched again.  A face dimension padded by 32
 *   unused columns (n_face = 32,800 instead of 32,768, plane annular N = 7, FP32)
 *   removed 15 % of the HBM reads and 8 % of the flux launch time.
 *
 * Ownership: descriptor arrays are host memory owned by the caller and copied during
 * mortar_setup.  Face arrays passed to mortar_flux are device memory owned by the
 * caller; the library never frees or keeps them.  The handle owns its device buffers.
 *
 * Errors: every entry point returns MORTAR_OK (0) or a negative mortar_status; no
 * entry point aborts.  Calls on one handle must not overlap (one handle per stream).
 */
#ifndef MORTAR_H
#define MORTAR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MORTAR_OK = 0,
    MORTAR_ERR_INVALID_ARG = -1, /* bad descriptor, size, pointer, NaN/Inf displacement */
    MORTAR_ERR_UNSUPPORTED = -2, /* valid but not built (degree, node set, mode) */
    MORTAR_ERR_OOM = -3,         /* device or host allocation failed */
    MORTAR_ERR_HIP = -4,         /* a HIP runtime call failed */
    MORTAR_ERR_NOT_READY = -5    /* mortar_flux before the first displacement update */
} mortar_status;

/* Interface shapes of the paper's figure of 3D interface geometries: plane, plane annular
 * axial, and surfaces of revolution (cylindrical radial, conical). */
enum { MORTAR_GEOM_PLANE = 0, MORTAR_GEOM_ANNULUS = 1, MORTAR_GEOM_REVOLUTION = 2 };
enum { MORTAR_NODES_GAUSS = 0, MORTAR_NODES_LGL = 1 };
enum { MORTAR_EULER = 0, MORTAR_NAVIER_STOKES = 1 };
enum { MORTAR_FLUX_LF = 0, MORTAR_FLUX_ROE = 1 };
/* Element type of U, G, F: double for FP64, float for the others.  In the *_MFMA modes
 * the projections run on the matrix cores in bf16/fp16 with fp32 accumulation. */
enum { MORTAR_FP64 = 0, MORTAR_FP32 = 1, MORTAR_BF16_MFMA = 2, MORTAR_FP16_MFMA = 3 };

/* Description of one sliding interface (Sec. 4.3 index definitions). */
typedef struct mortar_iface_desc {
    int32_t geometry;         /* MORTAR_GEOM_*: informational; metrics decide the math */
    int32_t N;                /* polynomial degree, 1 <= N <= 15; N >= 10: FP64/FP32 only,
                                 VALU-projection kernel only, one launch per interface,
                                 flux arrays below 2 GiB (else UNSUPPORTED) */
    int32_t node_set;         /* MORTAR_NODES_*: Gauss or Gauss-Lobatto (Sec. 3.1) */
    int32_t n_par;            /* faces per side along the sliding direction (periodic) */
    int32_t n_perp;           /* faces per side across it */
    int32_t n_face_static;    /* columns of the static arrays (>= n_par * n_perp) */
    int32_t n_face_moving;    /* columns of the moving arrays */
    const int32_t *face_id_static; /* host [n_perp * n_par]: distinct columns */
    const int32_t *face_id_moving; /* host [n_perp * n_par]: distinct columns */
    const int32_t *owner_static;   /* host [n_perp * n_par] owner ranks r, or NULL (all 0) */
    const int32_t *owner_moving;   /* host [n_perp * n_par] owner ranks r~, or NULL */
    double l_par;             /* face length along the slide, in displacement units */
    double normal[3];         /* static-side unit normal when metrics == NULL */
    double dS;                /* surface element per reference area when metrics == NULL */
    const double *metrics;    /* host [4][P][n_face_static] or NULL (constant normal/dS) */
    int32_t physics;          /* MORTAR_EULER or MORTAR_NAVIER_STOKES */
    int32_t riemann;          /* MORTAR_FLUX_LF or MORTAR_FLUX_ROE */
    int32_t precision;        /* MORTAR_FP64, MORTAR_FP32, MORTAR_BF16_MFMA, MORTAR_FP16_MFMA */
    int32_t reserved;
    double gamma;             /* ratio of specific heats */
    double mu;                /* dynamic viscosity (NS) */
    double Pr;                /* Prandtl number (NS); the gas constant cancels in q.n */
} mortar_iface_desc;

typedef struct mortar_handle mortar_handle;

/* Validates n_iface descriptors without touching the GPU.  0 or INVALID_ARG/UNSUPPORTED. */
int mortar_validate(const mortar_iface_desc *desc, int n_iface);

/* Creates a handle for n_iface interfaces on the current HIP device: copies every
 * descriptor array, allocates device buffers (projection matrices, face tables, index
 * maps) and computes the FP64 node sets and mass matrices (Sec. 3.2: M depends only on
 * the basis).  *out is set only on success. */
int mortar_setup(const mortar_iface_desc *desc, int n_iface, mortar_handle **out);

/* Per-stage update (Sec. 4.3 and 4.4): for each interface i, Delta_i = disp[i] (host
 * array [n_iface]) is split into n = floor(Delta/l_par) and s = Delta/l_par - n in FP64
 * on the host.  When n mod n_par changed (or on the first call) the sorted index array A
 * and the map m are rebuilt on the device; the FP64 projection matrices for s are
 * assembled on the device every call.  Asynchronous on stream (a hipStream_t; NULL =
 * default stream); no allocation.  NaN/Inf displacement -> INVALID_ARG, nothing changed. */
int mortar_update_displacement(mortar_handle *h, const double *disp, void *stream);

/* Same with (n, s) given directly (host arrays [n_iface]), for displacements too large
 * for an FP64 quotient; requires 0 <= s < 1. */
int mortar_update_displacement_ns(mortar_handle *h, const int64_t *n, const double *s,
                                  void *stream);

/* The mortar flux of every interface (Sec. 3.3 steps 2-5).  Arrays of n_iface device
 * pointers: U_s[i], U_m[i] states, G_s[i], G_m[i] gradients (NULL entries, or NULL
 * arrays, for Euler), F_s[i], F_m[i] outputs, in the interface's element type.  Only
 * the interface's columns of F_s/F_m are written.  Inputs are not modified; outputs
 * must not alias inputs.  Asynchronous on stream; no allocation; graph-capturable.
 * NOT_READY before the first displacement update. */
int mortar_flux(mortar_handle *h, const void *const *U_s, const void *const *U_m,
                const void *const *G_s, const void *const *G_m, void *const *F_s,
                void *const *F_m, void *stream);

/* The BR1 lifting surface term of every interface: the gradients of the first
 * Bassi-Rebay method (Sec. 2) lift the interface average of the state, and on a sliding
 * interface that average passes through the same mortar operator as the flux (Sec. 3.3
 * steps 2-5, Sec. 4.1: the second pair of exchanges).  At every mortar node
 * U* = (U_static + U_moving) / 2 is formed, multiplied by each component of the static
 * normal and by the surface element, and projected back onto both sides' faces.
 * U_s[i], U_m[i]: states [5][P][n_face] as for mortar_flux; L_s[i], L_m[i]: outputs
 * [3][5][P][n_face] (component d, variable v, as the gradient inputs), the same values
 * on both sides (static normal; the caller applies the sign).  Only the interface's
 * columns are written.  One launch per interface: FP32 element type up to degree 9
 * through the register-direct body (projections on the matrix cores in FP32), otherwise
 * the VALU-projection kernel; in the bf16/fp16 modes it runs in FP32 (their element
 * type).  UNSUPPORTED when an output array reaches 2 GiB.  Asynchronous on stream; no allocation.  NOT_READY before
 * the first displacement update. */
int mortar_lifting(mortar_handle *h, const void *const *U_s, const void *const *U_m,
                   void *const *L_s, void *const *L_m, void *stream);

/* ---- one stage as a HIP graph (batched persistent launch, Sec. 4.4 multi-interface) --
 * mortar_graph_create captures the flux launch of every interface (one persistent
 * launch when the interfaces share element type, physics and flux) for the given fixed
 * device buffers (same conventions as mortar_flux) into an executable graph; it needs a
 * displacement already set.  mortar_graph_launch then runs one stage: the displacement
 * update of mortar_update_displacement (host split; index maps rebuilt on face crossings,
 * launched on stream before the graph) followed by the graph with the new fraction s
 * written into its kernel arguments.  The graph owns no face buffers; destroy it before
 * its handle.  Errors as for mortar_flux; a graph whose launch shape no longer fits
 * reports UNSUPPORTED. */
typedef struct mortar_graph mortar_graph;
int mortar_graph_create(mortar_handle *h, const void *const *U_s, const void *const *U_m,
                        const void *const *G_s, const void *const *G_m, void *const *F_s,
                        void *const *F_m, mortar_graph **out);
int mortar_graph_launch(mortar_graph *g, const double *disp, void *stream);
int mortar_graph_destroy(mortar_graph *g);

/* mortar_graph_create_cons: mortar_graph_create with the stage's conservation sums
 * (Sec. 3.2: both sides' integrals of the projected flux) in the same graph.  After the
 * flux launch(es) the graph computes what mortar_conservation_device(h, F_s, F_m, d_cons)
 * computes for those outputs, into d_cons ([n_iface][5][3] doubles in device memory,
 * owned by the caller and kept valid for the graph's lifetime).  mortar_graph_launch
 * then runs a whole stage (update, flux, conservation sums) with no host launch between
 * the flux and the sums.  Like mortar_conservation_device, the captured sums use the
 * handle's own partial-sum buffers: other calls of the handle on another stream that
 * overlap a replay race on them.  d_cons NULL: INVALID_ARG; otherwise errors as for
 * mortar_graph_create. */
int mortar_graph_create_cons(mortar_handle *h, const void *const *U_s, const void *const *U_m,
                             const void *const *G_s, const void *const *G_m, void *const *F_s,
                             void *const *F_m, double *d_cons, mortar_graph **out);

/* ---- launch tuning ----------------------------------------------------------------
 * How an interface's flux is launched.  variant: MORTAR_KERNEL_VALU (projections on the
 * vector units, tiles staged in LDS), MORTAR_KERNEL_MFMA_LDS (projections as matrix-core
 * GEMMs, tiles staged in LDS), MORTAR_KERNEL_REGISTER (one wave per tile, GEMM results
 * kept in registers; the only variant of the bf16/fp16 precisions), MORTAR_KERNEL_VALU_WIDE
 * (FP32 only: the VALU kernel with 72 KB of LDS, longer tiles), MORTAR_KERNEL_HYBRID
 * (FP32 only: tiles staged in LDS, both projections on the matrix cores over 16-face
 * chunks, pointwise fluxes on the vector units; not for the largest degrees with
 * metrics, whose tiles do not fit its LDS budget).  tile_len: output
 * faces per tile along the sliding direction (0 = the variant's largest; larger values
 * are capped to it).  grid: workgroups of the persistent launch (0 = every resident
 * slot of the device; otherwise at least 8, one per XCD).  Interfaces in one batched
 * launch share the VALU variant and the grid; each has its own tile_len.
 * Size limits (per array, bytes): the VALU, wide and hybrid variants need each flux array
 * below 2 GiB; the register variant needs every state, gradient, metric and flux array
 * at most 4 GiB - 256; MFMA_LDS has none, and an interface beyond the default variant's
 * limit is launched with it.  Degrees N >= 10 have only MORTAR_KERNEL_VALU.
 * mortar_set_tuning returns INVALID_ARG for a variant that cannot address the interface. */
enum { MORTAR_KERNEL_VALU = 0, MORTAR_KERNEL_MFMA_LDS = 1, MORTAR_KERNEL_REGISTER = 2,
       MORTAR_KERNEL_VALU_WIDE = 3, MORTAR_KERNEL_HYBRID = 4 };
typedef struct mortar_tuning {
    int32_t variant;
    int32_t tile_len;
    int32_t grid;
    int32_t reserved;       /* 0 */
} mortar_tuning;

/* Autotuner: times the candidate launches of every interface on the given buffers
 * (conventions of mortar_flux; F_s/F_m are overwritten) with HIP events on stream, reps
 * launches per candidate after one warm-up, and keeps the fastest.  Candidates: each
 * applicable variant with three tile lengths (single-interface launches), or three tile
 * lengths per interface and the grid (batched launch).  Needs a displacement already
 * set; synchronizes stream.  Allocates one 512 MiB device buffer for the duration of the
 * call and frees it before returning: it is filled before every timed launch so that the
 * inputs come from HBM (a stage with fresh data does not find them in the caches); if
 * that allocation fails the candidates are timed with warm caches.  A HIP error during
 * the timing returns HIP_ERROR with the handle's previous tuning restored.  Graphs
 * captured before a tuning change are refused by mortar_graph_launch (UNSUPPORTED):
 * capture them again. */
int mortar_autotune(mortar_handle *h, const void *const *U_s, const void *const *U_m,
                    const void *const *G_s, const void *const *G_m, void *const *F_s,
                    void *const *F_m, int reps, void *stream);

/* Current tuning of interface iface (host struct), and setting one (e.g. from a cache of
 * an earlier mortar_autotune).  INVALID_ARG for a variant the interface cannot use. */
int mortar_get_tuning(const mortar_handle *h, int iface, mortar_tuning *out);
int mortar_set_tuning(mortar_handle *h, int iface, const mortar_tuning *t);

/* Frees the handle and its device buffers (synchronizes the device first). */
int mortar_destroy(mortar_handle *h);

/* Static text for a status code. */
const char *mortar_error_string(int code);

/* The 1D node set the operator assumes for faces and mortars (ascending, host arrays
 * x[N+1], w[N+1] with the quadrature weights); Sec. 3.1: Legendre-Gauss or
 * Legendre-Gauss-Lobatto points.  Host only.  INVALID_ARG/UNSUPPORTED for bad N. */
int mortar_basis(int N, int node_set, double *x, double *w);

/* Host-side FP64 split of a displacement (the rule mortar_update_displacement uses). */
int mortar_decompose_displacement(double delta, double l_par, int64_t *n, double *s);

/* ---- inspection (synchronous; copy into caller-owned host buffers) ---------------- */

/* Current (n, s) of interface iface. */
int mortar_get_displacement(mortar_handle *h, int iface, int64_t *n, double *s);

/* Sorted index array A (host [5][2 * n_par * n_perp], rows (owner of the opposite face,
 * i_par, i_perp, i_sub, i_face), 0-based columns i_mortar) and inverse map m (host
 * [2][n_face] with m[i_sub][i_face] = i_mortar, -1 for columns not on the interface)
 * of one side (0 = static, 1 = moving), Sec. 4.4 and Appendix A. */
int mortar_get_index_map(mortar_handle *h, int iface, int side, int32_t *A, int32_t *m);

/* Static-to-moving pairing of the current displacement (Sec. 4.3, index relation
 * i~ = (i - n + i_sub - 1) mod n_par, 0-based, periodic): pair (host [2][n_par], caller
 * owned) gets pair[i_sub * n_par + i_par] = the moving face index along the slide that
 * mortar (i_par, i_sub) lies on, the same in every row.  Evaluated on the device by the
 * routine the index map is built from.  Synchronizes the device. */
int mortar_get_pairing(mortar_handle *h, int iface, int32_t *pair);

/* FP64 projection matrices of the current s: Pf[4][NP][NP] (mortar node, face node) and
 * Pb[4][NP][NP] (face node, mortar node); order: static i_sub 0, static i_sub 1, moving
 * i_sub 0 (upper part of the moving face), moving i_sub 1 (lower part). */
int mortar_get_projection(mortar_handle *h, int iface, double *Pf, double *Pb);

/* Conservation sums in FP64 (compensated): out (host [n_iface][5][3]) gets, per variable,
 * the static-side integral sum w_p w_q F, the moving-side one and the sum of |terms|.
 * When F_s/F_m are the outputs of the interface's last flux launch and that launch used
 * a VALU-projection kernel, the sums come from the per-workgroup partials it wrote (the
 * sums of exactly the values it stored); otherwise the flux arrays (device) are read.
 * Runs on stream and synchronizes it. */
int mortar_conservation(mortar_handle *h, const void *const *F_s, const void *const *F_m,
                        double *out, void *stream);

/* The same sums for every interface into a device array d_out [n_iface][5][3] (FP64),
 * asynchronously on stream: no synchronization, no allocation, graph-capturable.  This
 * is the per-stage form of the conservation residual (discrete conservation of the
 * mortar projections, Sec. 3.2); each interface's scratch is reused, so calls on one
 * handle must not overlap. */
int mortar_conservation_device(mortar_handle *h, const void *const *F_s, const void *const *F_m,
                               double *d_out, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): the sums of mortar_conservation_device
 * (same arguments and output, always by a pass over the flux arrays) with their partial
 * results in a static device array of the library instead of handle buffers.  Calls no
 * allocating routine.  At most 8 interfaces per handle (UNSUPPORTED beyond; 1.25 MiB of
 * partials, 160 KiB per interface, held on every device the library runs on until the
 * process ends).  Every call on one device shares that array: calls that overlap on one
 * device (different streams, or handles used from several threads) race; calls on one
 * stream are ordered.  Every partial a call reads is written earlier in the same call, so
 * nothing needs clearing between calls.  Asynchronous on stream. */
int mortar_conservation_device_noalloc(mortar_handle *h, const void *const *F_s,
                                       const void *const *F_m, double *d_out, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* MORTAR_H */
