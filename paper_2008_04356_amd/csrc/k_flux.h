// Fused mortar-flux kernel: gather of both sides' face lines -> forward projection onto
// the two mortars of every static face -> Riemann + BR1 flux at every mortar node ->
// back projection onto the static and the moving faces (Sec. 3.3 steps 3-5 with the
// operators of Sec. 3.2).  One pass over HBM: every input value is read once (plus one
// halo face per tile), every output value is written once, mortar data stay in LDS.
//
// Work decomposition.  The tensor-product basis makes the operator act along the sliding
// direction only (Sec. 3.2: the problem splits into 1D operations along aligned lines),
// so every (row i_perp, line p_perp) is an independent periodic chain
//   ... (i-1, 1) (i, 0) (i, 1) (i+1, 0) ...
// of mortars: static face i owns (i, 0) and (i, 1); moving face i - n - 1 owns
// (i - 1, 1) and (i, 0).  A workgroup produces TF consecutive static faces i0 .. i0+TF-1
// and the TF moving faces i0-n-1 .. i0+TF-n-2 of one line.  It loads one halo face per
// side (static i0 - 1, moving i0+TF-n-1) and recomputes the halo mortar (i0 - 1, 1) that
// the first moving face needs; the neighbouring tile recomputes it as its own last
// mortar.  No atomics, deterministic.
//
// Phases (LDS-staged, 256 threads):
//   1. thread <-> (variable, face): coalesced loads of the NP values of a face line,
//      register mat-vec with both forward matrices, mortar values to LDS;
//   2. thread <-> mortar node: all variables of both sides from LDS, pointwise flux;
//   3. thread <-> (variable, face): the NP flux values of both mortars from LDS,
//      register mat-vec with both backward matrices, coalesced stores.
#pragma once

#include "flux_physics.h"
#include "mortar_internal.h"

namespace mortar {

template <typename T>
struct FluxArgs {
    const T *Us, *Um, *Gs, *Gm, *met;
    T *Fs, *Fm;
    const int32_t *fid_s, *fid_m;
    const char *params;          // ParamHeader + matrices
    int n_par, n_perp, nfs, nfm, tiles_per_row;
    T nx, ny, nz, dS;
    GasConsts<T> gas;
};

constexpr int kFluxThreads = 256;

// Faces per tile: the largest TF (<= 64) whose LDS footprint fits the budget.
template <typename T, int NP, int VS, int VM>
constexpr int tile_faces(int budget)
{
    int tf = 64;
    while (tf > 2 && (size_t)(VS + VM) * NP * (2 * tf + 2) * sizeof(T) > (size_t)budget) --tf;
    return tf;
}

template <typename T, int NP, bool NSV, bool MET, int RIEM, int BUDGET>
__global__ __launch_bounds__(kFluxThreads) void k_mortar_flux(FluxArgs<T> a)
{
    constexpr int V = NSV ? 20 : 5;          // projected values per side: U (+ 3x5 gradients)
    constexpr int VS = V + (MET ? 4 : 0);    // the static side also carries its metrics
    constexpr int TF = tile_faces<T, NP, VS, V>(BUDGET);
    constexpr int LD = 2 * TF + 2;           // LDS row: mortar slots of the tile
    constexpr int NN = NP * NP;
    constexpr int P = NN;
    constexpr int MAXPTS = (2 * TF + 1) * NP;
    constexpr int ROUNDS = (MAXPTS + kFluxThreads - 1) / kFluxThreads;
    static_assert((size_t)(VS + V) * NP * LD * sizeof(T) <= 160 * 1024, "LDS");

    __shared__ T lds[(VS + V) * NP * LD];
    T *ldsS = lds;                         // static values [VS][NP][LD], slot ms at column ms+1
    T *ldsM = lds + VS * NP * LD;          // moving values [V][NP][LD],  slot ms at column ms
    T *ldsF = lds;                         // fluxes [5][NP][LD] (reuses the static region)

    const int tid = threadIdx.x;
    const int t = blockIdx.x;
    const int chunk = t % a.tiles_per_row;
    const int rest = t / a.tiles_per_row;
    const int pp = rest % NP;              // line p_perp
    const int row = rest / NP;             // i_perp
    const int i0 = chunk * TF;
    const int nf = min(TF, a.n_par - i0);
    const int np_ = a.n_par;

    const ParamHeader *hdr = reinterpret_cast<const ParamHeader *>(a.params);
    const int nmod = hdr->nmod;
    const T *Pf = reinterpret_cast<const T *>(
        a.params + (sizeof(T) == 8 ? off_f64(NP) : off_f32(NP)));
    const T *Pb = Pf + 4 * NN;

    const int32_t *fs_row = a.fid_s + (size_t)row * np_;
    const int32_t *fm_row = a.fid_m + (size_t)row * np_;
    const size_t plane_s = (size_t)P * a.nfs, plane_m = (size_t)P * a.nfm;

    // ---- phase 1: gather and forward projection -----------------------------------
    constexpr int NIT_S = VS * (TF + 1);
    constexpr int NIT_M = V * (TF + 1);
    for (int it = tid; it < NIT_S + NIT_M; it += kFluxThreads) {
        if (it < NIT_S) {
            const int v = it / (TF + 1);
            const int f = it - v * (TF + 1);        // slot 0 = halo face i0 - 1
            if (f > nf) continue;
            int i = i0 - 1 + f;
            if (i < 0) i += np_;
            const int col = fs_row[i];
            const T *src = v < 5 ? a.Us + v * plane_s
                         : (v < V ? a.Gs + (v - 5) * plane_s : a.met + (v - V) * plane_s);
            T u[NP];
#pragma unroll
            for (int j = 0; j < NP; ++j) u[j] = src[(size_t)(j + NP * pp) * a.nfs + col];
#pragma unroll
            for (int q = 0; q < NP; ++q) {
                T q0 = T(0), q1 = T(0);
#pragma unroll
                for (int j = 0; j < NP; ++j) {
                    q0 += Pf[0 * NN + q * NP + j] * u[j];
                    q1 += Pf[1 * NN + q * NP + j] * u[j];
                }
                T *dst = ldsS + (v * NP + q) * LD;
                if (f >= 1) dst[2 * f] = q0;       // mortar (i, 0): slot 2f - 1
                dst[2 * f + 1] = q1;               // mortar (i, 1): slot 2f
            }
        } else {
            const int e = it - NIT_S;
            const int v = e / (TF + 1);
            const int f = e - v * (TF + 1);        // slot nf: only its lower part is in the tile
            if (f > nf) continue;
            int jt = i0 + f - nmod - 1;            // moving face under mortars (i0+f-1,1),(i0+f,0)
            if (jt < 0) jt += np_;
            const int col = fm_row[jt];
            const T *src = v < 5 ? a.Um + v * plane_m : a.Gm + (v - 5) * plane_m;
            T u[NP];
#pragma unroll
            for (int j = 0; j < NP; ++j) u[j] = src[(size_t)(j + NP * pp) * a.nfm + col];
#pragma unroll
            for (int q = 0; q < NP; ++q) {
                T qu = T(0), ql = T(0);
#pragma unroll
                for (int j = 0; j < NP; ++j) {
                    qu += Pf[2 * NN + q * NP + j] * u[j];
                    ql += Pf[3 * NN + q * NP + j] * u[j];
                }
                T *dst = ldsM + (v * NP + q) * LD;
                dst[2 * f] = ql;                   // lower part: mortar (i0+f-1, 1), slot 2f
                dst[2 * f + 1] = qu;               // upper part: mortar (i0+f, 0),   slot 2f+1
            }
        }
    }
    __syncthreads();

    // ---- phase 2: flux at every mortar node ---------------------------------------
    const int nm = 2 * nf + 1;
    const int npts = nm * NP;
    T res[ROUNDS][5];
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
        const int pt = tid + r * kFluxThreads;
        if (pt < npts) {
            const int q = pt / nm;
            const int ms = pt - q * nm;
            T UL[5], UR[5];
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                UL[v] = ldsS[(v * NP + q) * LD + ms + 1];
                UR[v] = ldsM[(v * NP + q) * LD + ms];
            }
            T nx = a.nx, ny = a.ny, nz = a.nz, dS = a.dS;
            if (MET) {
                nx = ldsS[((V + 0) * NP + q) * LD + ms + 1];
                ny = ldsS[((V + 1) * NP + q) * LD + ms + 1];
                nz = ldsS[((V + 2) * NP + q) * LD + ms + 1];
                dS = ldsS[((V + 3) * NP + q) * LD + ms + 1];
            }
            T F[5];
            convective_flux<T, RIEM>(UL, UR, nx, ny, nz, a.gas, F);
            if (NSV) {
                T G[15], FvL[5], FvR[5];
#pragma unroll
                for (int g = 0; g < 15; ++g) G[g] = ldsS[((5 + g) * NP + q) * LD + ms + 1];
                viscous_flux(UL, G, nx, ny, nz, a.gas, FvL);
#pragma unroll
                for (int g = 0; g < 15; ++g) G[g] = ldsM[((5 + g) * NP + q) * LD + ms];
                viscous_flux(UR, G, nx, ny, nz, a.gas, FvR);
#pragma unroll
                for (int v = 0; v < 5; ++v) F[v] -= T(0.5) * (FvL[v] + FvR[v]);
            }
#pragma unroll
            for (int v = 0; v < 5; ++v) res[r][v] = F[v] * dS;
        }
    }
    __syncthreads();   // the flux region overwrites static values still being read above
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
        const int pt = tid + r * kFluxThreads;
        if (pt < npts) {
            const int q = pt / nm;
            const int ms = pt - q * nm;
#pragma unroll
            for (int v = 0; v < 5; ++v) ldsF[(v * NP + q) * LD + ms] = res[r][v];
        }
    }
    __syncthreads();

    // ---- phase 3: back projection onto both sides ---------------------------------
    for (int it = tid; it < 10 * TF; it += kFluxThreads) {
        const int side = it >= 5 * TF;
        const int e = side ? it - 5 * TF : it;
        const int v = e / TF;
        const int f = e - v * TF;
        if (f >= nf) continue;
        const T *src = ldsF + v * NP * LD;
        T lo[NP], hi[NP];
        // static face i0+f: mortars (i0+f, 0) slot 2f+1 and (i0+f, 1) slot 2f+2
        // moving face i0+f-n-1: lower (i0+f-1, 1) slot 2f, upper (i0+f, 0) slot 2f+1
        const int s0 = side ? 2 * f : 2 * f + 1;
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            lo[q] = src[q * LD + s0];
            hi[q] = src[q * LD + s0 + 1];
        }
        const T *B_lo = Pb + (side ? 3 : 0) * NN;   // lower part's matrix
        const T *B_hi = Pb + (side ? 2 : 1) * NN;   // upper part's matrix
        T *dst;
        size_t stride;
        if (side) {
            int jt = i0 + f - nmod - 1;
            if (jt < 0) jt += np_;
            dst = a.Fm + v * plane_m + fm_row[jt];
            stride = a.nfm;
        } else {
            dst = a.Fs + v * plane_s + fs_row[i0 + f];
            stride = a.nfs;
        }
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            T acc = T(0);
#pragma unroll
            for (int q = 0; q < NP; ++q) acc += B_lo[j * NP + q] * lo[q] + B_hi[j * NP + q] * hi[q];
            dst[(size_t)(j + NP * pp) * stride] = acc;
        }
    }
}

}  // namespace mortar
