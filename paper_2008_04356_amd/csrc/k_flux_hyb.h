// Fused mortar-flux kernel with matrix-core projections (FP32 data, FP32 MFMA).
//
// The tile pipeline, LDS layout and pointwise flux phase of the VALU kernel (k_flux.h),
// with both projections of Sec. 3.2 done as 16x16x4 MFMA products instead of per-thread
// mat-vecs, which removes about two fifths of the vector instructions of a tile:
//   forward:  [Pf_a; Pf_b] (2NP x NP, rows interleaved: row 2q + 0 | 1 is node q of the
//             first | second mortar) times the face lines of 16 consecutive face slots of
//             one variable (K = face node, N = slot);
//   backward: [Pb_lo | Pb_hi] (NP x 2NP) times the fluxes of the two mortars of 16
//             consecutive faces (K = mortar node of lower | upper mortar, N = face).
// Matrix-core layouts (wave64, 16x16x4 f32): lane l holds A[l % 16][l / 16 + 4ks],
// B[l / 16 + 4ks][l % 16] and D[4 (l / 16) + r][l % 16], r = 0..3.  So every lane loads
// the values of one face slot (l % 16) at nodes l / 16 + 4ks: a tile has 16 NCH slots per
// side (TF = 16 NCH - 1 faces plus the halo), one face-column lookup per lane and chunk.
//
// Waves 0-1 take the static side, waves 2-3 the moving side, in phases 1 and 3 alike;
// wave w of a side takes the blocks (variable, chunk) b = w, w + 2, ...  As in the VALU
// kernel every lane issues every load and store (dead ones at valid or out-of-range
// addresses), so the compiler's memory waits stay exact.
#pragma once

#include "k_flux.h"

namespace mortar {

typedef float hyb_v4f __attribute__((ext_vector_type(4)));

// LDS budget per workgroup: three workgroups per CU.
constexpr int kLdsHyb = 53248;

// Tile capacity: the longest 16 n - 1 whose LDS fits the budget, 0 if none does.
template <int NP, int VS, int VM>
constexpr int pick_tile_hyb()
{
    int best = 0;
    for (int tf = 15; tf <= 63; tf += 16)
        if (tile_lds<float, NP, VS, VM>(tf) <= (size_t)kLdsHyb) best = tf;
    return best;
}

template <int NP, bool NSV, bool MET>
struct HybCfg {
    static constexpr int V = NSV ? 20 : 5;
    static constexpr int VS = V + (MET ? 4 : 0);
    static constexpr int NN = NP * NP;
    static constexpr int TF = pick_tile_hyb<NP, VS, V>();
    static constexpr int TFX = TF > 0 ? TF : 15;                 // keeps dead instantiations well formed
    static constexpr int LD = 2 * TFX + 4;
    static constexpr int NCH = (TFX + 1) / 16;                  // 16-slot chunks
    static constexpr int KS = (NP + 3) / 4;                     // K steps, forward
    static constexpr int MB = (2 * NP + 15) / 16;               // 16-row blocks, forward
    static constexpr int KS3 = (2 * NP + 3) / 4;                // K steps, backward
    static constexpr int NB_S = VS * NCH, NB_M = V * NCH;       // forward blocks per side
    static constexpr int NBW = ((NB_S > NB_M ? NB_S : NB_M) + 1) / 2;   // per wave
    static constexpr int NB3 = 5 * NCH;                         // backward blocks per side
    static constexpr int NB3W = (NB3 + 1) / 2;
    static constexpr int ROUNDS = ((2 * TFX + 1) * NP + kFluxThreads - 1) / kFluxThreads;
    static constexpr int LDS_T = (VS + V) * NP * LD;
};

template <int NP, bool NSV, bool MET>
constexpr size_t hyb_smem_bytes()
{
    using C = HybCfg<NP, NSV, MET>;
    return ((size_t)C::LDS_T * sizeof(float) + 15) / 16 * 16 + (size_t)8 * C::NN * sizeof(float);
}

template <int NP, bool NSV, bool MET, int RIEM>
__device__ __forceinline__ void run_interface_hyb(const FluxArgs<float> &a, TileCursor &cur, char *smem)
{
    using C = HybCfg<NP, NSV, MET>;
    using T = float;
    constexpr int V = C::V, VS = C::VS, NN = C::NN, TF = C::TFX, LD = C::LD, NCH = C::NCH;
    constexpr int KS = C::KS, MB = C::MB, KS3 = C::KS3, NBW = C::NBW, NB3W = C::NB3W;
    static_assert(C::LDS_T * sizeof(T) >= assemble_scratch<NP>() * sizeof(double), "assembly scratch");
    static_assert(NP <= 16, "one 16-row block of face nodes in the back projection");

    T *lds = reinterpret_cast<T *>(smem);
    T *mats = reinterpret_cast<T *>(smem + ((size_t)C::LDS_T * sizeof(T) + 15) / 16 * 16);
    T *ldsS = lds;                          // static values [VS][NP][LD], slot ms at column ms+1
    T *ldsM = lds + VS * NP * LD;           // moving values [V][NP][LD],  slot ms at column ms
    T *ldsF = lds;                          // fluxes [5][NP][LD] (reuses the static region)

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int c16 = lane & 15, g4 = lane >> 4;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int side = wave >> 1;             // 0: static, 1: moving
    const int w2 = wave & 1;
    const int np_ = a.n_par;
    const size_t plane_s = (size_t)NN * a.nfs, plane_m = (size_t)NN * a.nfm;
    const size_t stride = side ? a.nfm : a.nfs;
    const int nb1 = side ? C::NB_M : C::NB_S;
    const int32_t *fid = side ? a.fid_m : a.fid_s;
    const buf_rsrc_t rF = side ? buf_rsrc(a.Fm, (uint32_t)(5 * plane_m * sizeof(T)))
                               : buf_rsrc(a.Fs, (uint32_t)(5 * plane_s * sizeof(T)));
    const uint32_t nfo = side ? a.nfm : a.nfs;

    // face column of slot f (phase 1: static face i0-1+f, moving face i0+f-n-1) and of
    // output face f (phase 3: static face i0+f, moving face i0+f-n-1), clamped to the tile
    auto in_col = [&](const TileGeom &g, int f) {
        int i = g.i0 + min(f, g.nf) + (side ? -a.nmod - 1 : -1);
        if (i < 0) i += np_;
        return fid[(size_t)g.row * np_ + i];
    };
    auto out_col = [&](const TileGeom &g, int f) {
        int i = g.i0 + min(f, g.nf - 1) + (side ? -a.nmod - 1 : 0);
        if (i < 0) i += np_;
        return fid[(size_t)g.row * np_ + i];
    };
    // forward-block loads of one tile: block b = w2 + 2 kb, variable b / NCH, chunk b % NCH
    auto prefetch = [&](const TileGeom &g, const int (&col)[NCH], T (&u)[NBW][KS]) {
#pragma unroll
        for (int kb = 0; kb < NBW; ++kb) {
            const int b = min(w2 + 2 * kb, nb1 - 1);           // dead blocks reload the last
            const int v = b / NCH, ch = b - (b / NCH) * NCH;
            const T *src = !side ? (v < 5 ? a.Us + v * plane_s
                                          : (v < V ? a.Gs + (v - 5) * plane_s : a.met + (v - V) * plane_s))
                                 : (v < 5 ? a.Um + v * plane_m : a.Gm + (v - 5) * plane_m);
            src += col[ch] + (size_t)NP * g.pp * stride;
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int j = 4 * ks + g4;
                u[kb][ks] = src[(size_t)(j < NP ? j : 0) * stride];
            }
        }
    };

    // Pipeline as in the VALU kernel: tile t+1 loads during tile t; input columns of tile
    // t+2 and output columns of tile t+1 looked up at the start of tile t.
    TileGeom g = tile_geom(a, cur.tile(), NP);
    cur.next();
    bool more = cur.valid();
    TileGeom gn = tile_geom(a, more ? cur.tile() : 0, NP);
    T u[NBW][KS];
    int col[NCH], col_n[NCH], col3[NCH], col3_n[NCH];
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) col[ch] = in_col(g, 16 * ch + c16);
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) col3[ch] = out_col(g, 16 * ch + c16);
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch) col_n[ch] = in_col(gn, 16 * ch + c16);
    prefetch(g, col, u);
    // stores that write nothing, in the place of the previous tile's (see the VALU kernel)
#pragma unroll
    for (int k = 0; k < NB3W * 4; ++k) buf_store<T>(T(0), rF, kBufOff + (uint32_t)(k * sizeof(T)), 0);

    assemble_matrices<NP, T>(a.basis, a.s, reinterpret_cast<double *>(lds), nullptr, nullptr,
                             mats, mats + 4 * NN);

    // matrix-core A operands of this wave's side, kept in registers
    T A1[MB][KS], A3[KS3];
    {
        const T *PA = mats + (side ? 3 : 0) * NN;
        const T *PB = mats + (side ? 2 : 1) * NN;
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int m = 16 * mb + c16, k = 4 * ks + g4;
                const T *Pm = (m & 1) ? PB : PA;
                A1[mb][ks] = (m < 2 * NP && k < NP) ? Pm[(m >> 1) * NP + k] : T(0);
            }
        const T *Blo = mats + 4 * NN + (side ? 3 : 0) * NN;
        const T *Bhi = mats + 4 * NN + (side ? 2 : 1) * NN;
#pragma unroll
        for (int ks = 0; ks < KS3; ++ks) {
            const int j = c16, k = 4 * ks + g4;
            A3[ks] = (j < NP && k < 2 * NP) ? (k < NP ? Blo[j * NP + k] : Bhi[j * NP + k - NP]) : T(0);
        }
    }

    while (true) {
        cur.next();
        const bool more2 = cur.valid();
        const TileGeom gnn = tile_geom(a, more2 ? cur.tile() : 0, NP);
        int col_nn[NCH];
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) col_nn[ch] = in_col(gnn, 16 * ch + c16);
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) col3_n[ch] = out_col(gn, 16 * ch + c16);

        // ---- phase 1: forward projection on the matrix cores ------------------------
        {
            T *base = side ? ldsM : ldsS;
            typedef T T2 __attribute__((ext_vector_type(2)));
#pragma unroll
            for (int kb = 0; kb < NBW; ++kb) {
                const int b = w2 + 2 * kb;
                if (b < nb1) {                                  // uniform over the wave
                    const int v = b / NCH, ch = b - (b / NCH) * NCH;
                    const int f = 16 * ch + c16;                // slot, <= TF
                    hyb_v4f d[MB];
#pragma unroll
                    for (int mb = 0; mb < MB; ++mb) d[mb] = hyb_v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int ks = 0; ks < KS; ++ks) {
                        const T bv = 4 * ks + g4 < NP ? u[kb][ks] : T(0);
#pragma unroll
                        for (int mb = 0; mb < MB; ++mb)
                            d[mb] = __builtin_amdgcn_mfma_f32_16x16x4f32(A1[mb][ks], bv, d[mb], 0, 0, 0);
                    }
                    // rows 4 g4 + r of block mb: node q = 8 mb + 2 g4 + r / 2, mortar r % 2
#pragma unroll
                    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                        for (int h = 0; h < 2; ++h) {
                            const int q = 8 * mb + 2 * g4 + h;
                            if (q < NP)
                                *reinterpret_cast<T2 *>(base + (v * NP + q) * LD + 2 * f) =
                                    T2{d[mb][2 * h], d[mb][2 * h + 1]};
                        }
                }
            }
        }
        // the next tile's loads fly while this tile's flux and back projection run
        prefetch(gn, col_n, u);
        __syncthreads();

        // ---- phase 2: flux at every mortar node -------------------------------------
        flux_points<T, NP, NSV, MET, RIEM, LD, C::ROUNDS>(a, g.nf, ldsS, ldsM, ldsF);

        // ---- phase 3: back projection on the matrix cores ---------------------------
        // static face i0+f: mortars (i0+f, 0) slot 2f+1 and (i0+f, 1) slot 2f+2
        // moving face i0+f-n-1: lower (i0+f-1, 1) slot 2f, upper (i0+f, 0) slot 2f+1
#pragma unroll
        for (int kb = 0; kb < NB3W; ++kb) {
            const int b = min(w2 + 2 * kb, C::NB3 - 1);
            const bool live = w2 + 2 * kb < C::NB3;
            const int v = b / NCH, ch = b - (b / NCH) * NCH;
            const int f = 16 * ch + c16;                        // face, <= TF
            const T *src = ldsF + v * NP * LD + (side ? 2 * f : 2 * f + 1);
            hyb_v4f d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int ks = 0; ks < KS3; ++ks) {
                const int k = 4 * ks + g4;
                const T bv = k < NP ? src[k * LD] : (k < 2 * NP ? src[(k - NP) * LD + 1] : T(0));
                d = __builtin_amdgcn_mfma_f32_16x16x4f32(A3[ks], bv, d, 0, 0, 0);
            }
            const bool ok = live && f < g.nf;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int j = 4 * g4 + r;
                const uint32_t off = ((uint32_t)(v * NN + min(j, NP - 1) + NP * g.pp) * nfo + (uint32_t)col3[ch]) *
                                     (uint32_t)sizeof(T);
                buf_store<T>(d[r], rF, ok && j < NP ? off : kBufOff, 0);
            }
        }
        __syncthreads();   // phase 3 reads the LDS that the next phase 1 overwrites
        if (!more) break;
        g = gn;
        gn = gnn;
        more = more2;
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            col_n[ch] = col_nn[ch];
            col3[ch] = col3_n[ch];
        }
    }
}

template <int NP, bool NSV, bool MET, int RIEM>
__global__ __launch_bounds__(kFluxThreads) void k_mortar_flux_hyb(FluxArgs<float> a)
{
    if constexpr (HybCfg<NP, NSV, MET>::TF == 0) {
        return;                              // no tile fits: the host never launches it
    } else {
        __shared__ __attribute__((aligned(16))) char smem[hyb_smem_bytes<NP, NSV, MET>()];
        TileCursor cur(a.n_tiles);
        if (!cur.valid()) return;            // uniform over the workgroup
        run_interface_hyb<NP, NSV, MET, RIEM>(a, cur, smem);
    }
}

}  // namespace mortar
