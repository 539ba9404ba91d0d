// Fused mortar-flux kernel with the projections on the matrix cores.
//
// Same operator and the same tile chain as the VALU kernel (see k_flux.h), but both
// projections are small GEMMs over the 16 faces of a tile:
//   forward  (Sec. 3.2, face -> mortar):  Q[(sub, q)][f] = sum_j P_sub[q][j] U[j][f],
//            rows (sub-mortar, node) = 2 NP, K = face nodes NP, columns = 16 face slots;
//   backward (Sec. 3.2, mortar -> face):  F[j][f] = sum_k [B_lo | B_hi][j][k] Fm[k][f],
//            rows = face nodes NP, K = 2 NP mortar nodes of the face's two mortars.
// One v_mfma_*_16x16x4 per 4 of K (padded with zeros), accumulating in FP32 (FP64 for
// the FP64 path).  The matrix cores run these while the vector units evaluate the
// pointwise Riemann + BR1 fluxes of other waves, which stay on the VALU.
//
// A tile is one column group: static slots 0..15 = faces i0-1 .. i0+14 (slot 0 is the
// halo face), moving slots 0..15 = faces i0-n-1 .. i0+14-n; it produces up to 15 static
// and 15 moving faces.  The flux phase has (2 nf + 1) NP <= 31 NP mortar nodes, so a
// workgroup of about 32 NP threads evaluates them in one round.
#pragma once

#include "assemble.h"
#include "flux_physics.h"
#include "k_flux.h"
#include "mortar_internal.h"

namespace mortar {

typedef float mf_v4f __attribute__((ext_vector_type(4)));
typedef double mf_v4d __attribute__((ext_vector_type(4)));

// Operand lane layout of v_mfma_{f32,f64}_16x16x4 (A 16x4, B 4x16): lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16].  Result lane l, register r holds
// D[row][l % 16] with row = 4 (l / 16) + r for f32 and row = l / 16 + 4 r for f64.
template <typename T> struct Mma;
template <> struct Mma<float> {
    using acc = mf_v4f;
    __device__ static __forceinline__ acc mma(float a, float b, acc c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <> struct Mma<double> {
    using acc = mf_v4d;
    __device__ static __forceinline__ acc mma(double a, double b, acc c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};

template <typename T, int NP, bool NSV, bool MET>
struct MCfg {
    static constexpr int V = NSV ? 20 : 5;
    static constexpr int VS = V + (MET ? 4 : 0);
    static constexpr int NN = NP * NP;
    static constexpr int TF = 15;                        // output faces per tile
    static constexpr int LD = 2 * TF + 2;                // mortar slots per LDS row
    static constexpr int NT = ((2 * TF + 1) * NP + 63) / 64 * 64;
    static constexpr int NW = NT / 64;
    static constexpr int KS = (NP + 3) / 4;              // forward K steps
    static constexpr int RB = (2 * NP + 15) / 16;        // forward row blocks
    static constexpr int KS3 = (2 * NP + 3) / 4;         // backward K steps
    static constexpr int TASKS = VS + V;                 // forward tasks: one per variable and side
    static constexpr int TPW = (TASKS + NW - 1) / NW;
    static constexpr int T3PW = (10 + NW - 1) / NW;      // backward tasks per wave
    static constexpr int LDS_T = (VS + V) * NP * LD;
};

template <typename T, int NP, bool NSV, bool MET, int RIEM>
__global__ __launch_bounds__((MCfg<T, NP, NSV, MET>::NT)) void k_mortar_flux_mfma(FluxArgs<T> a)
{
    using C = MCfg<T, NP, NSV, MET>;
    using M = Mma<T>;
    using acc_t = typename M::acc;
    constexpr int V = C::V, VS = C::VS, NN = C::NN, TF = C::TF, LD = C::LD, P = NN;
    constexpr int NT = C::NT, NW = C::NW, KS = C::KS, RB = C::RB, KS3 = C::KS3;
    static_assert(C::LDS_T * sizeof(T) >= assemble_scratch<NP>() * sizeof(double), "assembly scratch");

    __shared__ __attribute__((aligned(16))) T lds[C::LDS_T];
    __shared__ T mats[8 * NN];
    T *ldsS = lds;                          // static values [VS][NP][LD], slot ms at column ms+1
    T *ldsM = lds + VS * NP * LD;           // moving values [V][NP][LD],  slot ms at column ms
    T *ldsF = lds;                          // fluxes [5][NP][LD]

    TileCursor cur(a.n_tiles);
    if (!cur.valid()) return;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int col = lane & 15;              // face slot of this lane in the GEMMs
    const int kq = lane >> 4;               // K index within a step (A column / B row)
    const int np_ = a.n_par;
    const int nmod = a.nmod;
    const size_t plane_s = (size_t)P * a.nfs, plane_m = (size_t)P * a.nfm;

    // ---- forward loads of one tile: this wave's tasks, K steps; lane = (k, column) ----
    T b[C::TPW][KS];
    int col_s = 0, col_m = 0;               // face columns of this lane's slot
    auto load_tile = [&](const TileGeom &g) {
        int i = g.i0 - 1 + col;
        if (i < 0) i += np_;
        if (i >= np_) i -= np_;
        int jt = g.i0 + col - nmod - 1;
        if (jt < 0) jt += np_;
        if (jt >= np_) jt -= np_;
        const bool live = col <= g.nf;
        col_s = live ? a.fid_s[(size_t)g.row * np_ + i] : 0;
        col_m = live ? a.fid_m[(size_t)g.row * np_ + jt] : 0;
#pragma unroll
        for (int m = 0; m < C::TPW; ++m) {
            const int task = wave + NW * m;
            const bool mov = task >= VS;
            const int v = mov ? task - VS : task;
            const T *src;
            size_t stride;
            if (!mov) {
                src = (v < 5 ? a.Us + v * plane_s
                             : (v < V ? a.Gs + (v - 5) * plane_s : a.met + (v - V) * plane_s)) + col_s;
                stride = a.nfs;
            } else {
                src = (v < 5 ? a.Um + v * plane_m : a.Gm + (v - 5) * plane_m) + col_m;
                stride = a.nfm;
            }
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int j = kq + 4 * ks;
                const bool ok = task < C::TASKS && live && j < NP;
                b[m][ks] = ok ? src[(size_t)(j + NP * g.pp) * stride] : T(0);
            }
        }
    };

    TileGeom g = tile_geom(a, cur.tile(), NP);
    load_tile(g);

    assemble_matrices<NP, T>(a.basis, a.s, reinterpret_cast<double *>(lds), nullptr, nullptr,
                             mats, mats + 4 * NN);

    // A operands (matrices) of this lane, kept for the whole launch.
    //  forward, side s: rows 0..NP-1 = first part (static Pf0 / moving Pf3 (lower)),
    //                   rows NP..2NP-1 = second part (static Pf1 / moving Pf2 (upper))
    //  backward, side s: [B_lo | B_hi] = static [Pb0 | Pb1] / moving [Pb3 | Pb2]
    T Af[2][RB][KS], Ab[2][KS3];
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
        const T *Pa = mats + (sd ? 3 : 0) * NN;
        const T *Pz = mats + (sd ? 2 : 1) * NN;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int r = col + 16 * rb, k = kq + 4 * ks;
                T v = T(0);
                if (k < NP) {
                    if (r < NP) v = Pa[r * NP + k];
                    else if (r < 2 * NP) v = Pz[(r - NP) * NP + k];
                }
                Af[sd][rb][ks] = v;
            }
        const T *Bl = mats + 4 * NN + (sd ? 3 : 0) * NN;
        const T *Bh = mats + 4 * NN + (sd ? 2 : 1) * NN;
#pragma unroll
        for (int ks = 0; ks < KS3; ++ks) {
            const int j = col, k = kq + 4 * ks;
            T v = T(0);
            if (j < NP) {
                if (k < NP) v = Bl[j * NP + k];
                else if (k < 2 * NP) v = Bh[j * NP + (k - NP)];
            }
            Ab[sd][ks] = v;
        }
    }
    __syncthreads();   // mats are read; the state region is free again

    while (true) {
        // ---- phase 1: forward projections on the matrix cores -------------------------
#pragma unroll
        for (int m = 0; m < C::TPW; ++m) {
            const int task = wave + NW * m;
            if (task < C::TASKS) {
                const int mov = task >= VS;
                const int v = mov ? task - VS : task;
                T *dst = (mov ? ldsM : ldsS) + v * NP * LD;
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) {
                    acc_t d = {T(0), T(0), T(0), T(0)};
#pragma unroll
                    for (int ks = 0; ks < KS; ++ks) d = M::mma(Af[mov][rb][ks], b[m][ks], d);
                    if (col <= g.nf) {
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int row = M::row(lane, r) + 16 * rb;
                            if (row < NP) {
                                // static first part: slot 2f-1 (column 2f), not for the halo
                                if (mov || col >= 1) dst[row * LD + 2 * col] = d[r];
                            } else if (row < 2 * NP) {
                                dst[(row - NP) * LD + 2 * col + 1] = d[r];
                            }
                        }
                    }
                }
            }
        }
        cur.next();
        const bool more = cur.valid();
        TileGeom gn = g;
        if (more) {
            gn = tile_geom(a, cur.tile(), NP);
            load_tile(gn);
        }
        __syncthreads();

        // ---- phase 2: flux at every mortar node (VALU) ------------------------------
        const int nm = 2 * g.nf + 1;
        const int npts = nm * NP;
        T res[5];
        const int pt = tid;
        const bool has_pt = pt < npts;
        if (has_pt) {
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
                unit_normal(nx, ny, nz);
            }
            T F[5];
            convective_flux<T, RIEM>(UL, UR, nx, ny, nz, a.gas, F);
            if (NSV) {
                T G[15], FvL[5], FvR[5];
#pragma unroll
                for (int gg = 0; gg < 15; ++gg) G[gg] = ldsS[((5 + gg) * NP + q) * LD + ms + 1];
                viscous_flux(UL, G, nx, ny, nz, a.gas, FvL);
#pragma unroll
                for (int gg = 0; gg < 15; ++gg) G[gg] = ldsM[((5 + gg) * NP + q) * LD + ms];
                viscous_flux(UR, G, nx, ny, nz, a.gas, FvR);
#pragma unroll
                for (int v = 0; v < 5; ++v) F[v] -= T(0.5) * (FvL[v] + FvR[v]);
            }
#pragma unroll
            for (int v = 0; v < 5; ++v) res[v] = F[v] * dS;
        }
        __syncthreads();
        if (has_pt) {
            const int q = pt / nm;
            const int ms = pt - q * nm;
#pragma unroll
            for (int v = 0; v < 5; ++v) ldsF[(v * NP + q) * LD + ms] = res[v];
        }
        __syncthreads();

        // ---- phase 3: back projections on the matrix cores --------------------------
        {
            const int32_t *fs_row = a.fid_s + (size_t)g.row * np_;
            const int32_t *fm_row = a.fid_m + (size_t)g.row * np_;
            const bool live = col < g.nf;
            int outc_s = 0, outc_m = 0;
            if (live) {
                outc_s = fs_row[g.i0 + col];
                int jt = g.i0 + col - nmod - 1;
                if (jt < 0) jt += np_;
                outc_m = fm_row[jt];
            }
#pragma unroll
            for (int m = 0; m < C::T3PW; ++m) {
                const int task = wave + NW * m;
                if (task < 10) {
                    const int sd = task >= 5;
                    const int v = sd ? task - 5 : task;
                    const T *src = ldsF + v * NP * LD;
                    // static face i0+f: lower part slot 2f+1, upper 2f+2;
                    // moving face i0+f-n-1: lower 2f, upper 2f+1
                    const int s0 = sd ? 2 * col : 2 * col + 1;
                    acc_t d = {T(0), T(0), T(0), T(0)};
#pragma unroll
                    for (int ks = 0; ks < KS3; ++ks) {
                        const int k = kq + 4 * ks;
                        T bv = T(0);
                        if (live && k < 2 * NP)
                            bv = k < NP ? src[k * LD + s0] : src[(k - NP) * LD + s0 + 1];
                        d = M::mma(Ab[sd][ks], bv, d);
                    }
                    if (live) {
                        T *dst = sd ? a.Fm + v * plane_m + outc_m : a.Fs + v * plane_s + outc_s;
                        const size_t stride = sd ? a.nfm : a.nfs;
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int j = M::row(lane, r);
                            if (j < NP) dst[(size_t)(j + NP * g.pp) * stride] = d[r];
                        }
                    }
                }
            }
        }
        if (!more) break;
        __syncthreads();
        g = gn;
    }
}

}  // namespace mortar
