// Pointwise interface fluxes of the compressible Navier-Stokes equations in conservative
// variables U = (rho, rho u, rho v, rho w, rho E) (Sec. 2 of arXiv 2008.04356):
//   - Roe's approximate Riemann solver with the Harten-Hyman entropy fix on the two
//     acoustic fields (Sec. 3.1), or the local Lax-Friedrichs flux;
//   - the BR1 viscous flux, the mean of both sides' viscous normal fluxes, with Stokes'
//     hypothesis lambda = -2/3 mu and Fourier heat flux q = -k grad T (Sec. 2);
//   - no grid-velocity term: on a sliding interface the grid moves tangentially, so
//     v_g . n vanishes.
// Everything is computed in the static side's normal direction and multiplied by the
// surface element.
#pragma once

#include <hip/hip_runtime.h>

namespace mortar {

template <typename T>
struct GasConsts {
    T gm1;    // gamma - 1
    T gamma;
    T mu;
    T kfac;   // mu * gamma / ((gamma - 1) Pr): heat conduction coefficient over R
};

// FP32 uses the hardware reciprocal and square root (about 1 ulp, well inside the FP32
// tolerance); FP64 keeps IEEE division and square root.
template <typename T> __device__ __forceinline__ T dsqrt(T x);
template <> __device__ __forceinline__ float dsqrt<float>(float x) { return __builtin_amdgcn_sqrtf(x); }
template <> __device__ __forceinline__ double dsqrt<double>(double x) { return __builtin_sqrt(x); }
template <typename T> __device__ __forceinline__ T drcp(T x);
template <> __device__ __forceinline__ float drcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ __forceinline__ double drcp<double>(double x) { return 1.0 / x; }

template <typename T> __device__ __forceinline__ T drsqrt(T x);
template <> __device__ __forceinline__ float drsqrt<float>(float x) { return __builtin_amdgcn_rsqf(x); }
template <> __device__ __forceinline__ double drsqrt<double>(double x) { return 1.0 / __builtin_sqrt(x); }

// Per-point metrics: on a curved face the interpolant of the unit nodal normals is
// shorter than one between the nodes, so the flux takes its direction scaled to unit
// length.  (On a flat face this changes nothing beyond rounding.)
template <typename T>
__device__ __forceinline__ void unit_normal(T &nx, T &ny, T &nz) {
    const T s = drsqrt<T>(nx * nx + ny * ny + nz * nz);
    nx *= s;
    ny *= s;
    nz *= s;
}

template <typename T> __device__ __forceinline__ T dabs(T x) { return x < T(0) ? -x : x; }
template <typename T> __device__ __forceinline__ T dmax(T a, T b) { return a > b ? a : b; }

// Primitive state of one side and its physical normal flux.
template <typename T>
struct Side {
    T r, ir, u[3], p, vn, H, c;
    T F[5];
};

template <typename T>
__device__ __forceinline__ void side_state(const T *U, T nx, T ny, T nz, const GasConsts<T> &g,
                                           Side<T> &o)
{
    o.r = U[0];
    o.ir = drcp(o.r);
    o.u[0] = U[1] * o.ir;
    o.u[1] = U[2] * o.ir;
    o.u[2] = U[3] * o.ir;
    const T kin = T(0.5) * (U[1] * o.u[0] + U[2] * o.u[1] + U[3] * o.u[2]);
    o.p = g.gm1 * (U[4] - kin);
    o.vn = o.u[0] * nx + o.u[1] * ny + o.u[2] * nz;
    o.H = (U[4] + o.p) * o.ir;
    o.c = dsqrt(g.gamma * o.p * o.ir);
    o.F[0] = U[0] * o.vn;
    o.F[1] = U[1] * o.vn + o.p * nx;
    o.F[2] = U[2] * o.vn + o.p * ny;
    o.F[3] = U[3] * o.vn + o.p * nz;
    o.F[4] = o.H * o.F[0];
}

// Harten-Hyman: inside a sonic expansion of width delta the eigenvalue modulus is
// replaced by the smooth (lambda^2/delta + delta)/2.
template <typename T>
__device__ __forceinline__ T entropy_fixed(T lam, T lamL, T lamR)
{
    const T delta = dmax(T(0), dmax(lam - lamL, lamR - lam));
    const T a = dabs(lam);
    return (a < delta) ? T(0.5) * (lam * lam * drcp(delta) + delta) : a;
}

// Convective numerical flux of two sides whose primitive states are already formed,
// RIEM = 0: local Lax-Friedrichs, 1: Roe + Harten-Hyman.
template <typename T, int RIEM>
__device__ __forceinline__ void convective_flux_sides(const Side<T> &L, const Side<T> &R,
                                                      const T *UL, const T *UR, T nx, T ny, T nz,
                                                      const GasConsts<T> &g, T *F)
{
    if (RIEM == 0) {
        const T lam = dmax(dabs(L.vn) + L.c, dabs(R.vn) + R.c);
#pragma unroll
        for (int v = 0; v < 5; ++v) F[v] = T(0.5) * ((L.F[v] + R.F[v]) - lam * (UR[v] - UL[v]));
        return;
    }
    // Roe averages with sqrt(rho) weights
    const T sl = dsqrt(L.r), sr = dsqrt(R.r);
    const T iw = drcp(sl + sr);
    const T wl = sl * iw, wr = sr * iw;
    T u[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) u[d] = wl * L.u[d] + wr * R.u[d];
    const T H = wl * L.H + wr * R.H;
    const T q2h = T(0.5) * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    const T c2 = g.gm1 * (H - q2h);
    const T c = dsqrt(c2);
    const T ic2 = drcp(c2);
    const T rho = sl * sr;
    const T un = u[0] * nx + u[1] * ny + u[2] * nz;
    // jumps
    const T dr = R.r - L.r, dp = R.p - L.p;
    T du[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) du[d] = R.u[d] - L.u[d];
    const T dun = du[0] * nx + du[1] * ny + du[2] * nz;
    // acoustic strengths and the entropy-wave strength
    const T rcdun = rho * c * dun;
    const T a1 = T(0.5) * (dp - rcdun) * ic2;
    const T a5 = T(0.5) * (dp + rcdun) * ic2;
    const T a2 = dr - dp * ic2;
    const T m1 = entropy_fixed(un - c, L.vn - L.c, R.vn - R.c) * a1;
    const T m5 = entropy_fixed(un + c, L.vn + L.c, R.vn + R.c) * a5;
    const T m2 = dabs(un);
    // tangential velocity jump (shear waves)
    T dt[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) dt[d] = du[d] - dun * (d == 0 ? nx : (d == 1 ? ny : nz));
    const T sum15 = m1 + m5;
    const T dif15 = (m5 - m1) * c;
    const T D0 = sum15 + m2 * a2;
    const T rm2 = rho * m2;
    T D[5];
    D[0] = D0;
    D[1] = D0 * u[0] + dif15 * nx + rm2 * dt[0];
    D[2] = D0 * u[1] + dif15 * ny + rm2 * dt[1];
    D[3] = D0 * u[2] + dif15 * nz + rm2 * dt[2];
    D[4] = sum15 * H + dif15 * un + m2 * a2 * q2h + rm2 * (u[0] * dt[0] + u[1] * dt[1] + u[2] * dt[2]);
#pragma unroll
    for (int v = 0; v < 5; ++v) F[v] = T(0.5) * ((L.F[v] + R.F[v]) - D[v]);
}

// Convective numerical flux, RIEM = 0: local Lax-Friedrichs, 1: Roe + Harten-Hyman.
template <typename T, int RIEM>
__device__ __forceinline__ void convective_flux(const T *UL, const T *UR, T nx, T ny, T nz,
                                                const GasConsts<T> &g, T *F)
{
    Side<T> L, R;
    side_state(UL, nx, ny, nz, g, L);
    side_state(UR, nx, ny, nz, g, R);
    convective_flux_sides<T, RIEM>(L, R, UL, UR, nx, ny, nz, g, F);
}

// Viscous normal flux Fv(U, grad U) . n of one side from its 1/rho, velocity and p/rho;
// G[d*5 + v] = dU_v/dx_d.
template <typename T>
__device__ __forceinline__ void viscous_flux_prim(const T ir, const T v0, const T v1, const T v2,
                                                  const T p_over_r, const T *G, T nx, T ny, T nz,
                                                  const GasConsts<T> &g, T *Fv)
{
    const T half_v2 = T(0.5) * (v0 * v0 + v1 * v1 + v2 * v2);
    T gv[3][3];   // gv[i][d] = d v_i / d x_d
    T kgT[3];     // k dT/dx_d divided by nothing more: includes the gas-constant cancellation
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const T *Gd = G + 5 * d;
        gv[0][d] = (Gd[1] - v0 * Gd[0]) * ir;
        gv[1][d] = (Gd[2] - v1 * Gd[0]) * ir;
        gv[2][d] = (Gd[3] - v2 * Gd[0]) * ir;
        const T dp = g.gm1 * (Gd[4] - (v0 * Gd[1] + v1 * Gd[2] + v2 * Gd[3]) + half_v2 * Gd[0]);
        kgT[d] = g.kfac * (dp - p_over_r * Gd[0]) * ir;
    }
    // traction tau n = mu ((grad v + grad v^T) n - 2/3 (div v) n), mu factored out
    const T div23 = T(-2.0 / 3.0) * (gv[0][0] + gv[1][1] + gv[2][2]);
    const T nn[3] = {nx, ny, nz};
    T tn[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        T a = div23 * nn[i];
#pragma unroll
        for (int j = 0; j < 3; ++j) a += (gv[i][j] + gv[j][i]) * nn[j];
        tn[i] = g.mu * a;
    }
    Fv[0] = T(0);
    Fv[1] = tn[0];
    Fv[2] = tn[1];
    Fv[3] = tn[2];
    Fv[4] = v0 * tn[0] + v1 * tn[1] + v2 * tn[2] + kgT[0] * nx + kgT[1] * ny + kgT[2] * nz;
}

// Viscous normal flux Fv(U, grad U) . n of one side; G[d*5 + v] = dU_v/dx_d.
template <typename T>
__device__ __forceinline__ void viscous_flux(const T *U, const T *G, T nx, T ny, T nz,
                                             const GasConsts<T> &g, T *Fv)
{
    const T ir = drcp(U[0]);
    const T v0 = U[1] * ir, v1 = U[2] * ir, v2 = U[3] * ir;
    const T half_v2 = T(0.5) * (v0 * v0 + v1 * v1 + v2 * v2);
    viscous_flux_prim(ir, v0, v1, v2, g.gm1 * (U[4] * ir - half_v2), G, nx, ny, nz, g, Fv);
}

// The same from the primitive state convective_flux_sides used (the side's 1/rho,
// velocity and pressure are not formed again).
template <typename T>
__device__ __forceinline__ void viscous_flux_side(const Side<T> &S, const T *G, T nx, T ny, T nz,
                                                  const GasConsts<T> &g, T *Fv)
{
    viscous_flux_prim(S.ir, S.u[0], S.u[1], S.u[2], S.p * S.ir, G, nx, ny, nz, g, Fv);
}

}  // namespace mortar
