// A small DGSEM solver for the compressible Euler / Navier-Stokes equations on a periodic
// Cartesian box
// whose central slab slides along x1 (Sec. 5.2 of arXiv 2008.04356: the convergence test
// of the sliding-mesh method on a planar interface).  It exists to embed the mortar
// operator of libmortar.so in a whole scheme: the two sliding planes get their fluxes
// from that operator (called by the driver), every other face from the Lax-Friedrichs
// flux here.  C ABI in include/dg_embed.h.
//
// Discretization (Sec. 3.1): Legendre-Gauss nodes, tensor-product Lagrange basis, weak
// form with the diagonal Gauss mass matrix; on an element of edge h, per direction d
//   dU_i/dt = (2/h) [ sum_m Dw[i][m] F_d(U_m) - (l_i(+1) F*_+ - l_i(-1) F*_-) / w_i ],
//   Dw[i][m] = (w_m / w_i) l_i'(x_m),
// summed over the three directions.  In the moving slab the flux is the ALE flux
// F - vg U e1 (Sec. 2); the grid velocity is tangential to the sliding planes.
// Navier-Stokes (Sec. 2, first Bassi-Rebay method): the gradients are lifted with the
// average of both sides' states on every face (the sliding planes' averages come from the
// mortar operator's lifting term),
//   Q_i = (2/h) [ (l_i(+1) U*_+ - l_i(-1) U*_-) / w_i - sum_m Dw[i][m] U_m ],
// the flux is F_c - F_v(U, Q), and the viscous face flux the average of both sides'.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "dg_embed.h"
#include "flux_physics.h"

namespace dgembed {

constexpr int kMaxNP = 8;

// Table layout (doubles): x[NP], w[NP], lm[NP] = l_j(-1), lp[NP] = l_j(+1), Dw[NP][NP].
__host__ __device__ inline int tab_doubles(int NP) { return 4 * NP + NP * NP; }

struct Tab {
    const double *x, *w, *lm, *lp, *Dw;
    __device__ Tab(const double *b, int NP)
        : x(b), w(b + NP), lm(b + 2 * NP), lp(b + 3 * NP), Dw(b + 4 * NP) {}
};

struct Geo {
    int NP, K, j_lo, j_hi;
    double h, L, vg, gm1, gamma, rho0, amp, u0, p0;
    bool ns;
    mortar::GasConsts<double> gas;   // gamma - 1, gamma, mu, k / R
};

inline Geo geo(const dg_grid &g)
{
    Geo o;
    o.NP = g.N + 1;
    o.K = g.K;
    o.j_lo = g.j_lo;
    o.j_hi = g.j_hi;
    o.L = g.L;
    o.h = g.L / g.K;
    o.vg = g.vg;
    o.gamma = g.gamma;
    o.gm1 = g.gamma - 1.0;
    o.rho0 = g.rho0;
    o.amp = g.amp;
    o.u0 = g.u0;
    o.p0 = g.p0;
    o.ns = g.mu > 0.0;
    o.gas = {o.gm1, o.gamma, o.ns ? g.mu : 0.0, o.ns ? g.mu * g.gamma / (o.gm1 * g.Pr) : 0.0};
    return o;
}

__device__ inline bool moving_layer(const Geo &G, int j) { return j >= G.j_lo && j < G.j_hi; }

// Euler flux in direction d of state U.
__device__ inline void euler_flux(const double *U, int d, double gm1, double *F)
{
    const double ir = 1.0 / U[0];
    const double ud = U[1 + d] * ir;
    const double p = gm1 * (U[4] - 0.5 * (U[1] * U[1] + U[2] * U[2] + U[3] * U[3]) * ir);
    F[0] = U[1 + d];
    F[1] = U[1] * ud;
    F[2] = U[2] * ud;
    F[3] = U[3] * ud;
    F[1 + d] += p;
    F[4] = (U[4] + p) * ud;
}

// Lax-Friedrichs flux in direction +e_d between UL (below) and UR (above), with the
// grid velocity component vgn along e_d: 1/2 (F_L + F_R) - 1/2 vgn (UL + UR)
// - 1/2 lambda (UR - UL), lambda = max over both sides of |u_d - vgn| + c.
__device__ inline void lf_flux(const double *UL, const double *UR, int d, double vgn,
                               const Geo &G, double *F)
{
    double FL[5], FR[5];
    euler_flux(UL, d, G.gm1, FL);
    euler_flux(UR, d, G.gm1, FR);
    auto speed = [&](const double *U) {
        const double ir = 1.0 / U[0];
        const double p = G.gm1 * (U[4] - 0.5 * (U[1] * U[1] + U[2] * U[2] + U[3] * U[3]) * ir);
        return fabs(U[1 + d] * ir - vgn) + sqrt(G.gamma * p * ir);
    };
    const double lam = fmax(speed(UL), speed(UR));
#pragma unroll
    for (int v = 0; v < 5; ++v)
        F[v] = 0.5 * (FL[v] + FR[v]) - 0.5 * vgn * (UL[v] + UR[v]) - 0.5 * lam * (UR[v] - UL[v]);
}

__device__ inline int elem(const Geo &G, int i, int j, int k) { return i + G.K * (j + G.K * k); }
__device__ inline int wrap(int i, int K) { return i < 0 ? i + K : (i >= K ? i - K : i); }

// Node of direction d's line through face point (p, q) of a face normal to d, at
// position m along d.
__device__ inline int line_node(int NP, int d, int m, int p, int q)
{
    if (d == 0) return m + NP * (p + NP * q);     // face point (b, c)
    if (d == 1) return p + NP * (m + NP * q);     // face point (a, c)
    return p + NP * (q + NP * m);                 // face point (a, b)
}

// Value of variable v of element e on its face in direction d (side: 0 = -, 1 = +) at
// face point (p, q): the element polynomial evaluated at -1 / +1 along d.
__device__ inline double face_value(const double *U, const Tab &T, int NP, int e, int v, int d,
                                    int side, int p, int q)
{
    const double *l = side ? T.lp : T.lm;
    const double *u = U + ((size_t)e * 5 + v) * NP * NP * NP;
    double s = 0.0;
    for (int m = 0; m < NP; ++m) s += l[m] * u[line_node(NP, d, m, p, q)];
    return s;
}

__global__ void k_exact(Geo G, const double *tab, double t, double *U)
{
    const int NP = G.NP, NN = NP * NP * NP;
    const int n_elem = G.K * G.K * G.K;
    const Tab T(tab, NP);
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < n_elem * NN; idx += gridDim.x * blockDim.x) {
        const int e = idx / NN, node = idx % NN;
        const int i = e % G.K, j = (e / G.K) % G.K, k = e / (G.K * G.K);
        const int a = node % NP, b = (node / NP) % NP, c = node / (NP * NP);
        double x1 = (i + 0.5 * (T.x[a] + 1.0)) * G.h;
        const double x2 = (j + 0.5 * (T.x[b] + 1.0)) * G.h;
        const double x3 = (k + 0.5 * (T.x[c] + 1.0)) * G.h;
        if (moving_layer(G, j)) x1 += G.vg * t;
        const double ph = 2.0 * M_PI * (x1 + x2 + x3 - 3.0 * G.u0 * t) / G.L;
        const double rho = G.rho0 + G.amp * sin(ph);
        double *u = U + (size_t)e * 5 * NN + node;
        u[0 * NN] = rho;
        u[1 * NN] = rho * G.u0;
        u[2 * NN] = rho * G.u0;
        u[3 * NN] = rho * G.u0;
        u[4 * NN] = G.p0 / G.gm1 + 0.5 * rho * 3.0 * G.u0 * G.u0;
    }
}

// Value of lifted gradient (d2, v) of element e on its face in direction d.
__device__ inline double face_grad(const double *Q, const Tab &T, int NP, int e, int d2, int v, int d,
                                   int side, int p, int q)
{
    const double *l = side ? T.lp : T.lm;
    const double *u = Q + (((size_t)e * 3 + d2) * 5 + v) * NP * NP * NP;
    double s = 0.0;
    for (int m = 0; m < NP; ++m) s += l[m] * u[line_node(NP, d, m, p, q)];
    return s;
}

// One thread per (direction, element, face point) of the + face of each element.
__global__ void k_faces(Geo G, const double *tab, const double *U, const double *Q, double *FF)
{
    const int NP = G.NP, NF = NP * NP;
    const int n_elem = G.K * G.K * G.K;
    const Tab T(tab, NP);
    const int total = 3 * n_elem * NF;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += gridDim.x * blockDim.x) {
        const int d = idx / (n_elem * NF);
        const int rest = idx % (n_elem * NF);
        const int e = rest / NF, fp = rest % NF;
        const int p = fp % NP, q = fp / NP;
        const int i = e % G.K, j = (e / G.K) % G.K, k = e / (G.K * G.K);
        // the sliding planes are the mortar operator's
        if (d == 1 && (j == G.j_lo - 1 || j == G.j_hi - 1)) continue;
        const int en = d == 0 ? elem(G, wrap(i + 1, G.K), j, k)
                     : d == 1 ? elem(G, i, wrap(j + 1, G.K), k) : elem(G, i, j, wrap(k + 1, G.K));
        double UL[5], UR[5], F[5];
        for (int v = 0; v < 5; ++v) {
            UL[v] = face_value(U, T, NP, e, v, d, 1, p, q);
            UR[v] = face_value(U, T, NP, en, v, d, 0, p, q);
        }
        const double vgn = (d == 0 && moving_layer(G, j)) ? G.vg : 0.0;
        lf_flux(UL, UR, d, vgn, G, F);
        if (Q) {
            // first Bassi-Rebay: minus the average of both sides' viscous fluxes
            double GL[15], GR[15], FvL[5], FvR[5];
            for (int d2 = 0; d2 < 3; ++d2)
                for (int v = 0; v < 5; ++v) {
                    GL[d2 * 5 + v] = face_grad(Q, T, NP, e, d2, v, d, 1, p, q);
                    GR[d2 * 5 + v] = face_grad(Q, T, NP, en, d2, v, d, 0, p, q);
                }
            const double nx = d == 0, ny = d == 1, nz = d == 2;
            mortar::viscous_flux(UL, GL, nx, ny, nz, G.gas, FvL);
            mortar::viscous_flux(UR, GR, nx, ny, nz, G.gas, FvR);
            for (int v = 0; v < 5; ++v) F[v] -= 0.5 * (FvL[v] + FvR[v]);
        }
        double *o = FF + (((size_t)d * n_elem + e) * 5) * NF + fp;
        for (int v = 0; v < 5; ++v) o[v * NF] = F[v];
    }
}

// The average of both sides' states on the + face of every element (conforming faces).
__global__ void k_face_states(Geo G, const double *tab, const double *U, double *UF)
{
    const int NP = G.NP, NF = NP * NP;
    const int n_elem = G.K * G.K * G.K;
    const Tab T(tab, NP);
    const int total = 3 * n_elem * NF;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += gridDim.x * blockDim.x) {
        const int d = idx / (n_elem * NF);
        const int rest = idx % (n_elem * NF);
        const int e = rest / NF, fp = rest % NF;
        const int p = fp % NP, q = fp / NP;
        const int i = e % G.K, j = (e / G.K) % G.K, k = e / (G.K * G.K);
        if (d == 1 && (j == G.j_lo - 1 || j == G.j_hi - 1)) continue;
        const int en = d == 0 ? elem(G, wrap(i + 1, G.K), j, k)
                     : d == 1 ? elem(G, i, wrap(j + 1, G.K), k) : elem(G, i, j, wrap(k + 1, G.K));
        double *o = UF + (((size_t)d * n_elem + e) * 5) * NF + fp;
        for (int v = 0; v < 5; ++v)
            o[v * NF] = 0.5 * (face_value(U, T, NP, e, v, d, 1, p, q) + face_value(U, T, NP, en, v, d, 0, p, q));
    }
}

// Lifted gradients: one workgroup per element, one thread per node.
template <int NP>
__global__ __launch_bounds__(512) void k_gradients(Geo G, const double *tab, const double *U,
                                                   const double *UF, const double *Ls0, const double *Lm0,
                                                   const double *Ls1, const double *Lm1, double *Q)
{
    constexpr int NN = NP * NP * NP, NF = NP * NP;
    __shared__ double u[5][NN];
    const Tab T(tab, NP);
    const int n_elem = G.K * G.K * G.K, KK = G.K * G.K;
    const int e = blockIdx.x;
    const int i = e % G.K, j = (e / G.K) % G.K, k = e / (G.K * G.K);
    const int node = threadIdx.x;
    const bool live = node < NN;
    if (live)
        for (int v = 0; v < 5; ++v) u[v][node] = U[((size_t)e * 5 + v) * NN + node];
    __syncthreads();
    if (!live) return;
    const int a = node % NP, b = (node / NP) % NP, c = node / NF;
    const int e0m = elem(G, wrap(i - 1, G.K), j, k);
    const int e1m = elem(G, i, wrap(j - 1, G.K), k);
    const int e2m = elem(G, i, j, wrap(k - 1, G.K));
    const int col = i + G.K * k;
    const double s = 2.0 / G.h;
    for (int v = 0; v < 5; ++v) {
        double d0 = 0.0, d1 = 0.0, d2 = 0.0;
#pragma unroll
        for (int m = 0; m < NP; ++m) {
            d0 += T.Dw[a * NP + m] * u[v][m + NP * (b + NP * c)];
            d1 += T.Dw[b * NP + m] * u[v][a + NP * (m + NP * c)];
            d2 += T.Dw[c * NP + m] * u[v][a + NP * (b + NP * m)];
        }
        const double u0p = UF[(((size_t)0 * n_elem + e) * 5 + v) * NF + b + NP * c];
        const double u0m = UF[(((size_t)0 * n_elem + e0m) * 5 + v) * NF + b + NP * c];
        const int fp2 = a + NP * c;
        // the sliding planes: component 2 (the e2 normal) of the operator's lifting term
        const size_t li = ((size_t)(1 * 5 + v) * NF + fp2) * KK + col;
        double u1p, u1m;
        if (j == G.j_lo - 1) u1p = Ls0[li];
        else if (j == G.j_hi - 1) u1p = Ls1[li];
        else u1p = UF[(((size_t)1 * n_elem + e) * 5 + v) * NF + fp2];
        if (j == G.j_lo) u1m = Lm0[li];
        else if (j == G.j_hi) u1m = Lm1[li];
        else u1m = UF[(((size_t)1 * n_elem + e1m) * 5 + v) * NF + fp2];
        const double u2p = UF[(((size_t)2 * n_elem + e) * 5 + v) * NF + a + NP * b];
        const double u2m = UF[(((size_t)2 * n_elem + e2m) * 5 + v) * NF + a + NP * b];
        double *o = Q + ((size_t)e * 3 * 5 + v) * NN + node;
        o[0 * 5 * NN] = s * ((T.lp[a] * u0p - T.lm[a] * u0m) / T.w[a] - d0);
        o[1 * 5 * NN] = s * ((T.lp[b] * u1p - T.lm[b] * u1m) / T.w[b] - d1);
        o[2 * 5 * NN] = s * ((T.lp[c] * u2p - T.lm[c] * u2m) / T.w[c] - d2);
    }
}

// Face gradients of both sliding planes for the mortar operator ([3][5][NP^2][K^2] each).
__global__ void k_prolong_grad(Geo G, const double *tab, const double *Q, double *Gs0, double *Gm0,
                               double *Gs1, double *Gm1)
{
    const int NP = G.NP, NF = NP * NP, KK = G.K * G.K;
    const Tab T(tab, NP);
    const int total = 2 * KK * NF;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += gridDim.x * blockDim.x) {
        const int itf = idx / (KK * NF);
        const int rest = idx % (KK * NF);
        const int col = rest / NF, fp = rest % NF;
        const int i = col % G.K, k = col / G.K;
        const int a = fp % NP, c = fp / NP;
        const int jb = itf == 0 ? G.j_lo - 1 : G.j_hi - 1;
        const int eb = elem(G, i, jb, k), ea = elem(G, i, jb + 1, k);
        double *Gs = itf == 0 ? Gs0 : Gs1, *Gm = itf == 0 ? Gm0 : Gm1;
        for (int d2 = 0; d2 < 3; ++d2)
            for (int v = 0; v < 5; ++v) {
                const size_t o = ((size_t)(d2 * 5 + v) * NF + fp) * KK + col;
                Gs[o] = face_grad(Q, T, NP, eb, d2, v, 1, 1, a, c);
                Gm[o] = face_grad(Q, T, NP, ea, d2, v, 1, 0, a, c);
            }
    }
}

// Face states of both sliding planes for the mortar operator ([5][NP^2][K^2] each).
__global__ void k_prolong(Geo G, const double *tab, const double *U, double *Us0, double *Um0,
                          double *Us1, double *Um1)
{
    const int NP = G.NP, NF = NP * NP, KK = G.K * G.K;
    const Tab T(tab, NP);
    const int total = 2 * KK * NF;
    for (int idx = blockIdx.x * blockDim.x + threadIdx.x; idx < total; idx += gridDim.x * blockDim.x) {
        const int itf = idx / (KK * NF);
        const int rest = idx % (KK * NF);
        const int col = rest / NF, fp = rest % NF;
        const int i = col % G.K, k = col / G.K;
        const int a = fp % NP, c = fp / NP;
        const int jb = itf == 0 ? G.j_lo - 1 : G.j_hi - 1;   // layer below the plane
        const int eb = elem(G, i, jb, k), ea = elem(G, i, jb + 1, k);
        double *Us = itf == 0 ? Us0 : Us1, *Um = itf == 0 ? Um0 : Um1;
        for (int v = 0; v < 5; ++v) {
            Us[((size_t)v * NF + fp) * KK + col] = face_value(U, T, NP, eb, v, 1, 1, a, c);
            Um[((size_t)v * NF + fp) * KK + col] = face_value(U, T, NP, ea, v, 1, 0, a, c);
        }
    }
}

// The energy source that makes the travelling density wave a Navier-Stokes solution: its
// velocity is uniform (no stress) and its pressure constant, so only the heat flux is
// left: S = -div(k grad T) = -(k/R) p0 laplacian(1/rho), with rho(phi), phi = kappa (x1 +
// x2 + x3 - 3 u0 t), kappa = 2 pi / L: laplacian(1/rho) = 3 kappa^2 (1/rho)''(phi),
// (1/rho)'' = -rho''/rho^2 + 2 rho'^2/rho^3.
__device__ inline double energy_source(const Geo &G, const Tab &T, int i, int j, int k, int a, int b,
                                       int c, double t)
{
    double x1 = (i + 0.5 * (T.x[a] + 1.0)) * G.h;
    const double x2 = (j + 0.5 * (T.x[b] + 1.0)) * G.h;
    const double x3 = (k + 0.5 * (T.x[c] + 1.0)) * G.h;
    if (moving_layer(G, j)) x1 += G.vg * t;
    const double kappa = 2.0 * M_PI / G.L;
    const double ph = kappa * (x1 + x2 + x3 - 3.0 * G.u0 * t);
    const double rho = G.rho0 + G.amp * sin(ph);
    const double r1 = G.amp * cos(ph), r2 = -G.amp * sin(ph);
    const double inv2 = -r2 / (rho * rho) + 2.0 * r1 * r1 / (rho * rho * rho);
    return -G.gas.kfac * G.p0 * 3.0 * kappa * kappa * inv2;
}

// Volume and surface terms: one workgroup per element, one thread per node.
template <int NP>
__global__ __launch_bounds__(512) void k_rhs(Geo G, const double *tab, const double *U, const double *Q,
                                             const double *FF, const double *Fs0, const double *Fm0,
                                             const double *Fs1, const double *Fm1, double t, double *dU)
{
    constexpr int NN = NP * NP * NP, NF = NP * NP;
    __shared__ double f[3][5][NN];
    const Tab T(tab, NP);
    const int n_elem = G.K * G.K * G.K, KK = G.K * G.K;
    const int e = blockIdx.x;
    const int i = e % G.K, j = (e / G.K) % G.K, k = e / (G.K * G.K);
    const int node = threadIdx.x;
    const bool live = node < NN;
    const int a = node % NP, b = (node / NP) % NP, c = node / NF;
    const bool mov = moving_layer(G, j);
    if (live) {
        double u[5];
        for (int v = 0; v < 5; ++v) u[v] = U[((size_t)e * 5 + v) * NN + node];
        double gq[15];
        if (Q)
            for (int d2 = 0; d2 < 3; ++d2)
                for (int v = 0; v < 5; ++v) gq[d2 * 5 + v] = Q[(((size_t)e * 3 + d2) * 5 + v) * NN + node];
        for (int d = 0; d < 3; ++d) {
            double F[5];
            euler_flux(u, d, G.gm1, F);
            if (d == 0 && mov)
                for (int v = 0; v < 5; ++v) F[v] -= G.vg * u[v];
            if (Q) {
                double Fv[5];
                mortar::viscous_flux(u, gq, (double)(d == 0), (double)(d == 1), (double)(d == 2), G.gas, Fv);
                for (int v = 0; v < 5; ++v) F[v] -= Fv[v];
            }
            for (int v = 0; v < 5; ++v) f[d][v][node] = F[v];
        }
    }
    __syncthreads();
    if (!live) return;
    const int e0m = elem(G, wrap(i - 1, G.K), j, k);
    const int e1m = elem(G, i, wrap(j - 1, G.K), k);
    const int e2m = elem(G, i, j, wrap(k - 1, G.K));
    const int col = i + G.K * k;
    const double s = 2.0 / G.h;
    for (int v = 0; v < 5; ++v) {
        double r = 0.0;
#pragma unroll
        for (int m = 0; m < NP; ++m) {
            r += T.Dw[a * NP + m] * f[0][v][m + NP * (b + NP * c)];
            r += T.Dw[b * NP + m] * f[1][v][a + NP * (m + NP * c)];
            r += T.Dw[c * NP + m] * f[2][v][a + NP * (b + NP * m)];
        }
        // x1 faces
        const double f0p = FF[(((size_t)0 * n_elem + e) * 5 + v) * NF + b + NP * c];
        const double f0m = FF[(((size_t)0 * n_elem + e0m) * 5 + v) * NF + b + NP * c];
        // x2 faces: the sliding planes take the mortar operator's fluxes
        const int fp2 = a + NP * c;
        double f1p, f1m;
        if (j == G.j_lo - 1) f1p = Fs0[((size_t)v * NF + fp2) * KK + col];
        else if (j == G.j_hi - 1) f1p = Fs1[((size_t)v * NF + fp2) * KK + col];
        else f1p = FF[(((size_t)1 * n_elem + e) * 5 + v) * NF + fp2];
        if (j == G.j_lo) f1m = Fm0[((size_t)v * NF + fp2) * KK + col];
        else if (j == G.j_hi) f1m = Fm1[((size_t)v * NF + fp2) * KK + col];
        else f1m = FF[(((size_t)1 * n_elem + e1m) * 5 + v) * NF + fp2];
        // x3 faces
        const double f2p = FF[(((size_t)2 * n_elem + e) * 5 + v) * NF + a + NP * b];
        const double f2m = FF[(((size_t)2 * n_elem + e2m) * 5 + v) * NF + a + NP * b];
        r -= (T.lp[a] * f0p - T.lm[a] * f0m) / T.w[a];
        r -= (T.lp[b] * f1p - T.lm[b] * f1m) / T.w[b];
        r -= (T.lp[c] * f2p - T.lm[c] * f2m) / T.w[c];
        r *= s;
        if (Q && v == 4) r += energy_source(G, T, i, j, k, a, b, c, t);
        dU[((size_t)e * 5 + v) * NN + node] = r;
    }
}

__global__ void k_rk(double *U, double *R, const double *dU, double a, double b, double dt, int64_t n)
{
    for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < n;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const double r = a * R[idx] + dt * dU[idx];
        R[idx] = r;
        U[idx] += b * r;
    }
}

__global__ void k_density_error(Geo G, const double *tab, const double *U, double t, double *err)
{
    const int NP = G.NP, NN = NP * NP * NP;
    const int n_elem = G.K * G.K * G.K;
    const Tab T(tab, NP);
    const double J = 0.125 * G.h * G.h * G.h;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n_elem; e += gridDim.x * blockDim.x) {
        const int i = e % G.K, j = (e / G.K) % G.K, k = e / (G.K * G.K);
        double acc = 0.0;
        for (int node = 0; node < NN; ++node) {
            const int a = node % NP, b = (node / NP) % NP, c = node / (NP * NP);
            double x1 = (i + 0.5 * (T.x[a] + 1.0)) * G.h;
            const double x2 = (j + 0.5 * (T.x[b] + 1.0)) * G.h;
            const double x3 = (k + 0.5 * (T.x[c] + 1.0)) * G.h;
            if (moving_layer(G, j)) x1 += G.vg * t;
            const double rho = G.rho0 + G.amp * sin(2.0 * M_PI * (x1 + x2 + x3 - 3.0 * G.u0 * t) / G.L);
            const double dr = U[(size_t)e * 5 * NN + node] - rho;
            acc += T.w[a] * T.w[b] * T.w[c] * J * dr * dr;
        }
        err[e] = acc;
    }
}

// ---- host: the degree's tables ------------------------------------------------------

// Legendre P_n and P_{n-1} by the three-term recurrence.
static void legendre(int n, double x, double &pn, double &pn1)
{
    double a = 1.0, b = x;
    if (n == 0) { pn = 1.0; pn1 = 0.0; return; }
    for (int k = 2; k <= n; ++k) {
        const double c = ((2 * k - 1) * x * b - (k - 1) * a) / k;
        a = b;
        b = c;
    }
    pn = b;
    pn1 = a;
}

// Gauss nodes by Newton's method from the Chebyshev-like initial guesses, weights from
// the derivative of P_np.
static void gauss(int np, double *x, double *w)
{
    for (int i = 0; i < np; ++i) {
        double t = -std::cos(M_PI * (i + 0.75) / (np + 0.5));
        for (int it = 0; it < 100; ++it) {
            double pn, pn1;
            legendre(np, t, pn, pn1);
            const double dp = np * (pn1 - t * pn) / ((1.0 - t) * (1.0 + t));
            const double dt = pn / dp;
            t -= dt;
            if (std::fabs(dt) < 1e-16) break;
        }
        double pn, pn1;
        legendre(np, t, pn, pn1);
        const double omx2 = (1.0 - t) * (1.0 + t);
        const double dp = np * (pn1 - t * pn) / omx2;
        x[i] = t;
        w[i] = 2.0 / (omx2 * dp * dp);
    }
}

}  // namespace dgembed

using namespace dgembed;

extern "C" {

int64_t dg_basis_bytes(int N)
{
    if (N < 1 || N + 1 > kMaxNP) return -1;
    return (int64_t)sizeof(double) * tab_doubles(N + 1);
}

int dg_basis_tables(int N, double *tab)
{
    if (!tab || N < 1 || N + 1 > kMaxNP) return -1;
    const int NP = N + 1;
    double *x = tab, *w = tab + NP, *lm = tab + 2 * NP, *lp = tab + 3 * NP, *Dw = tab + 4 * NP;
    gauss(NP, x, w);
    // Lagrange basis values at -1, +1 and derivatives at the nodes, from the product form
    auto lag = [&](int jj, double t) {
        double p = 1.0;
        for (int m = 0; m < NP; ++m)
            if (m != jj) p *= (t - x[m]) / (x[jj] - x[m]);
        return p;
    };
    auto dlag = [&](int jj, double t) {   // d/dt of l_jj at t (sum over the dropped factor)
        double s = 0.0;
        for (int r = 0; r < NP; ++r) {
            if (r == jj) continue;
            double p = 1.0 / (x[jj] - x[r]);
            for (int m = 0; m < NP; ++m)
                if (m != jj && m != r) p *= (t - x[m]) / (x[jj] - x[m]);
            s += p;
        }
        return s;
    };
    for (int jj = 0; jj < NP; ++jj) {
        lm[jj] = lag(jj, -1.0);
        lp[jj] = lag(jj, 1.0);
    }
    for (int ii = 0; ii < NP; ++ii)
        for (int m = 0; m < NP; ++m) Dw[ii * NP + m] = w[m] / w[ii] * dlag(ii, x[m]);
    return 0;
}

static bool grid_ok(const dg_grid *g)
{
    return g && g->N >= 1 && g->N + 1 <= kMaxNP && g->K >= 3 && g->j_lo > 0 && g->j_lo < g->j_hi &&
           g->j_hi < g->K && g->L > 0.0 && g->gamma > 1.0 && g->basis && g->mu >= 0.0 &&
           (g->mu == 0.0 || g->Pr > 0.0);
}

static int blocks_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 65536)); }

#define DG_TRY()                                       \
    do {                                               \
        if (hipGetLastError() != hipSuccess) return -4; \
    } while (0)

int dg_exact_state(const dg_grid *g, double t, double *U, void *stream)
{
    if (!grid_ok(g) || !U) return -1;
    const Geo G = geo(*g);
    const int64_t n = (int64_t)g->K * g->K * g->K * G.NP * G.NP * G.NP;
    hipLaunchKernelGGL(k_exact, dim3(blocks_for(n)), dim3(256), 0, (hipStream_t)stream, G, g->basis, t, U);
    DG_TRY();
    return 0;
}

int dg_face_fluxes(const dg_grid *g, const double *U, const double *Q, double *FF, void *stream)
{
    if (!grid_ok(g) || !U || !FF || (g->mu > 0.0) != (Q != nullptr)) return -1;
    const Geo G = geo(*g);
    const int64_t n = (int64_t)3 * g->K * g->K * g->K * G.NP * G.NP;
    hipLaunchKernelGGL(k_faces, dim3(blocks_for(n)), dim3(256), 0, (hipStream_t)stream, G, g->basis, U, Q, FF);
    DG_TRY();
    return 0;
}

int dg_face_states(const dg_grid *g, const double *U, double *UF, void *stream)
{
    if (!grid_ok(g) || !U || !UF) return -1;
    const Geo G = geo(*g);
    const int64_t n = (int64_t)3 * g->K * g->K * g->K * G.NP * G.NP;
    hipLaunchKernelGGL(k_face_states, dim3(blocks_for(n)), dim3(256), 0, (hipStream_t)stream, G, g->basis, U, UF);
    DG_TRY();
    return 0;
}

int dg_gradients(const dg_grid *g, const double *U, const double *UF, const double *Ls0,
                 const double *Lm0, const double *Ls1, const double *Lm1, double *Q, void *stream)
{
    if (!grid_ok(g) || !U || !UF || !Ls0 || !Lm0 || !Ls1 || !Lm1 || !Q) return -1;
    const Geo G = geo(*g);
    const int n_elem = g->K * g->K * g->K;
    const int NP = G.NP;
    const int threads = ((NP * NP * NP + 63) / 64) * 64;
    hipStream_t st = (hipStream_t)stream;
    switch (NP) {
#define DG_GRAD_CASE(np)                                                                      \
    case np:                                                                                  \
        hipLaunchKernelGGL(k_gradients<np>, dim3(n_elem), dim3(threads), 0, st, G, g->basis, U, UF, \
                           Ls0, Lm0, Ls1, Lm1, Q);                                            \
        break;
        DG_GRAD_CASE(2) DG_GRAD_CASE(3) DG_GRAD_CASE(4) DG_GRAD_CASE(5) DG_GRAD_CASE(6) DG_GRAD_CASE(7)
        DG_GRAD_CASE(8)
#undef DG_GRAD_CASE
    default: return -1;
    }
    DG_TRY();
    return 0;
}

int dg_prolong_interface_gradients(const dg_grid *g, const double *Q, double *Gs0, double *Gm0,
                                   double *Gs1, double *Gm1, void *stream)
{
    if (!grid_ok(g) || !Q || !Gs0 || !Gm0 || !Gs1 || !Gm1) return -1;
    const Geo G = geo(*g);
    const int64_t n = (int64_t)2 * g->K * g->K * G.NP * G.NP;
    hipLaunchKernelGGL(k_prolong_grad, dim3(blocks_for(n)), dim3(256), 0, (hipStream_t)stream, G, g->basis,
                       Q, Gs0, Gm0, Gs1, Gm1);
    DG_TRY();
    return 0;
}

int dg_prolong_interfaces(const dg_grid *g, const double *U, double *Us0, double *Um0,
                          double *Us1, double *Um1, void *stream)
{
    if (!grid_ok(g) || !U || !Us0 || !Um0 || !Us1 || !Um1) return -1;
    const Geo G = geo(*g);
    const int64_t n = (int64_t)2 * g->K * g->K * G.NP * G.NP;
    hipLaunchKernelGGL(k_prolong, dim3(blocks_for(n)), dim3(256), 0, (hipStream_t)stream, G, g->basis, U,
                       Us0, Um0, Us1, Um1);
    DG_TRY();
    return 0;
}

int dg_rhs(const dg_grid *g, const double *U, const double *Q, const double *FF,
           const double *Fs0, const double *Fm0, const double *Fs1, const double *Fm1, double t,
           double *dU, void *stream)
{
    if (!grid_ok(g) || !U || !FF || !Fs0 || !Fm0 || !Fs1 || !Fm1 || !dU) return -1;
    if ((g->mu > 0.0) != (Q != nullptr)) return -1;
    const Geo G = geo(*g);
    const int n_elem = g->K * g->K * g->K;
    const int NP = G.NP;
    const int threads = ((NP * NP * NP + 63) / 64) * 64;
    hipStream_t st = (hipStream_t)stream;
    switch (NP) {
#define DG_RHS_CASE(np)                                                                       \
    case np:                                                                                  \
        hipLaunchKernelGGL(k_rhs<np>, dim3(n_elem), dim3(threads), 0, st, G, g->basis, U, Q, FF,   \
                           Fs0, Fm0, Fs1, Fm1, t, dU);                                        \
        break;
        DG_RHS_CASE(2) DG_RHS_CASE(3) DG_RHS_CASE(4) DG_RHS_CASE(5) DG_RHS_CASE(6) DG_RHS_CASE(7)
        DG_RHS_CASE(8)
#undef DG_RHS_CASE
    default: return -1;
    }
    DG_TRY();
    return 0;
}

int dg_rk_stage(double *U, double *R, const double *dU, double a, double b, double dt, int64_t n,
                void *stream)
{
    if (!U || !R || !dU || n < 0) return -1;
    hipLaunchKernelGGL(k_rk, dim3(blocks_for(n)), dim3(256), 0, (hipStream_t)stream, U, R, dU, a, b, dt, n);
    DG_TRY();
    return 0;
}

int dg_density_error(const dg_grid *g, const double *U, double t, double *err, void *stream)
{
    if (!grid_ok(g) || !U || !err) return -1;
    const Geo G = geo(*g);
    const int n_elem = g->K * g->K * g->K;
    hipLaunchKernelGGL(k_density_error, dim3(blocks_for(n_elem)), dim3(256), 0, (hipStream_t)stream, G,
                       g->basis, U, t, err);
    DG_TRY();
    return 0;
}

}  // extern "C"
