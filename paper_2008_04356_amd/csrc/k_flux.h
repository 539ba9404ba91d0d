// Fused mortar-flux kernel: gather of both sides' face lines -> forward projection onto
// the two mortars of every static face -> Riemann + BR1 flux at every mortar node ->
// back projection onto the static and the moving faces (Sec. 3.3 steps 3-5 with the
// operators of Sec. 3.2).  One pass over HBM: every input value is read once (plus one
// halo face per side and tile), every output value is written once, mortar data stay in
// LDS.  One launch per stage: each workgroup assembles the FP64 projection matrices for
// the stage's fraction s itself while its first loads are in flight.
//
// Work decomposition.  The tensor-product basis makes the operator act along the sliding
// direction only (Sec. 3.2: the problem splits into 1D operations along aligned lines),
// so every (row i_perp, line p_perp) is an independent periodic chain
//   ... (i-1, 1) (i, 0) (i, 1) (i+1, 0) ...
// of mortars: static face i owns (i, 0) and (i, 1); moving face i - n - 1 owns
// (i - 1, 1) and (i, 0).  A workgroup produces the static faces i0 .. i0+nf-1 and the
// moving faces i0-n-1 .. i0+nf-n-2 of one line.  It loads one halo face per side
// (static i0 - 1, moving i0+nf-n-1) and recomputes the halo mortar (i0 - 1, 1) that the
// first moving face needs; the neighbouring tile recomputes it as its own last mortar.
// No atomics: results are deterministic.
//
// Phases (256 threads; threads 0-127 take the static side, 128-255 the moving side in
// phases 1 and 3):
//   0. every thread issues the global loads of all its face lines (register prefetch),
//      then the block assembles the FP64 matrices into LDS;
//   1. register mat-vec of each face line with the side's two forward matrices, mortar
//      values to LDS ([var][node][mortar slot], static slot ms at column ms + 1);
//   2. thread <-> mortar node: all variables of both sides from LDS, pointwise flux;
//   3. thread <-> (side, variable, face): the NP flux values of its two mortars from
//      LDS, mat-vec with the two backward matrices, coalesced stores.
#pragma once

#include "assemble.h"
#include "flux_physics.h"
#include "mortar_internal.h"

namespace mortar {

// Buffer access (bit patterns, no conversion) with a 32-bit per-lane byte offset and a
// scalar byte offset.  Word 3 of the descriptor: 32-bit data format, no swizzle, raw
// addressing; an access whose per-lane offset is at or beyond num_records bytes reads 0
// and writes nothing, which masks lanes without a branch.
typedef __amdgpu_buffer_rsrc_t buf_rsrc_t;
__device__ __forceinline__ buf_rsrc_t buf_rsrc(const void *p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}
template <typename T> __device__ __forceinline__ T buf_load(const buf_rsrc_t &r, uint32_t off, int soff);
template <> __device__ __forceinline__ float buf_load<float>(const buf_rsrc_t &r, uint32_t off, int soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, soff, 0));
}
template <> __device__ __forceinline__ double buf_load<double>(const buf_rsrc_t &r, uint32_t off, int soff)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, soff, 0));
}
typedef unsigned buf_u2 __attribute__((ext_vector_type(2)));
template <typename T> __device__ __forceinline__ void buf_store(T x, const buf_rsrc_t &r, uint32_t off, int soff);
template <> __device__ __forceinline__ void buf_store<float>(float x, const buf_rsrc_t &r, uint32_t off, int soff)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, (int)off, soff, 0);
}
template <> __device__ __forceinline__ void buf_store<double>(double x, const buf_rsrc_t &r, uint32_t off, int soff)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(buf_u2, x), r, (int)off, soff, 0);
}
// Per-lane offset of a masked-off lane: beyond every descriptor of the VALU kernel (its
// output arrays stay below 2 GiB).
constexpr uint32_t kBufOff = 0x80000000u;

template <typename T>
struct FluxArgs {
    const T *Us, *Um, *Gs, *Gm, *met;
    T *Fs, *Fm;
    const int32_t *fid_s, *fid_m;
    const BasisConsts *basis;
    double s;                     // sub-face fraction of the stage
    int nmod;                     // n mod n_par
    int n_par, n_perp, nfs, nfm;
    int tiles_per_row, tile_len;  // tile_len <= the compile-time tile capacity
    int n_tiles;                  // tiles_per_row * NP * n_perp
    T nx, ny, nz, dS;
    GasConsts<T> gas;
    // conservation partials of this launch, or null: the workgroup's FP64 sums of
    // w_p w_q F and w_p w_q |F| per (variable, side) group g = 2 v + side at
    // cons[(g * gridDim.x + blockIdx.x) * 2 + {0, 1}]
    double *cons;
};

// Compensated (Neumaier) FP64 sum.
struct ConsSum {
    double s = 0.0, c = 0.0;
    __device__ __forceinline__ void add(double x)
    {
        const double t = s + x;
        c += (fabs(s) >= fabs(x)) ? (s - t) + x : (x - t) + s;
        s = t;
    }
    __device__ __forceinline__ double value() const { return s + c; }
};

// Zero conservation partials of a workgroup that had no tile of the interface.
__device__ __forceinline__ void cons_zero(double *cons)
{
    if (cons && threadIdx.x < 20) cons[((size_t)(threadIdx.x >> 1) * gridDim.x + blockIdx.x) * 2 + (threadIdx.x & 1)] = 0.0;
}

constexpr int kFluxThreads = 256;
constexpr int kHalf = kFluxThreads / 2;
constexpr int kXcds = 8;   // MI355X: workgroups are dispatched round-robin over 8 XCDs

// LDS budget per workgroup of the VALU-projection kernel: 48 KB in FP32 (three
// workgroups per CU), 80 KB in FP64 (two).
template <typename T> constexpr int lds_budget() { return sizeof(T) == 8 ? 81920 : 49152; }
// The wide-tile FP32 instantiation: 72 KB, two workgroups per CU.
constexpr int kLdsWideF32 = 73728;

// Degree sets of the batched kernel: every degree, or the 1.5-stage turbine set N = 3, 5, 7.
constexpr int kMaskAll = 0x7FC;
constexpr int kMaskTurbine = (1 << 4) | (1 << 6) | (1 << 8);

// Persistent schedule over the n tiles of one interface.  Workgroup b runs on XCD b % 8
// (workgroups are dispatched round-robin over the XCDs); XCD x owns the contiguous eighth
// [x*ceil(n/8), (x+1)*ceil(n/8)) of the tiles and its workgroups take them in steps of
// the number of workgroups on that XCD.  So at any time the workgroups of one XCD work
// on neighbouring tiles of the same line (the cache lines a tile shares with its
// neighbours - halo faces, partial lines at its ends - are fetched into that XCD's L2
// once), and with several interfaces every XCD gets the same share of each.
struct TileCursor {
    int k, limit, stride;
    __device__ explicit TileCursor(int n)
    {
        const int g = gridDim.x;
        const int xcd = blockIdx.x % kXcds;
        const int local = blockIdx.x / kXcds;
        stride = g / kXcds + ((g % kXcds) > xcd ? 1 : 0);   // workgroups on this XCD
        const int per = (n + kXcds - 1) / kXcds;
        const int base = xcd * per;
        limit = min(n, base + per);
        k = base + local;
    }
    __device__ bool valid() const { return k < limit; }
    __device__ int tile() const { return k; }
    __device__ void next() { k += stride; }
};

// LDS bytes of a tile with capacity tf faces: per side, variable and node a row of 2 tf + 2
// mortar slots plus two columns that absorb the writes of dead projection items.
template <typename T, int NP, int VS, int VM>
constexpr size_t tile_lds(int tf)
{
    return (size_t)(VS + VM) * NP * (2 * tf + 4) * sizeof(T) + (size_t)8 * NP * NP * sizeof(T);
}

// Tile capacity: among the capacities whose LDS fits the budget, the one that best fills
// the 256-thread rounds of the flux phase, weighted by the halo overhead 1/(tf+1); or,
// for the wide-tile budget, simply the longest (per-tile costs dominate there).
template <typename T, int NP, int VS, int VM>
constexpr int pick_tile(int budget)
{
    int best = 2;
    double best_score = -1.0;
    for (int tf = 2; tf <= 64; ++tf) {
        if (tile_lds<T, NP, VS, VM>(tf) > (size_t)budget) break;
        const int pts = (2 * tf + 1) * NP;
        const int rounds = (pts + kFluxThreads - 1) / kFluxThreads;
        const double score = budget == kLdsWideF32 ? (double)tf
                                                   : (double)pts / (rounds * kFluxThreads) * tf / (tf + 1.0);
        if (score > best_score + 1e-9) {
            best_score = score;
            best = tf;
        }
    }
    return best;
}

// LIFT: the BR1 lifting surface term instead of the flux: states only in, 15 values
// (3 normal components x 5 variables) per point out.
template <typename T, int NP, bool NSV, bool MET, int BUDGET, bool LIFT = false>
struct FluxCfg {
    static constexpr int V = NSV ? 20 : 5;         // projected values per side
    static constexpr int VS = V + (MET ? 4 : 0);   // the static side also carries metrics
    static constexpr int NN = NP * NP;
    static constexpr int NOUT = LIFT ? 15 : 5;     // values per output point
    static constexpr int ROWS = VS + V > NOUT ? VS + V : NOUT;   // LDS rows of NP x LD
    static constexpr int TF = pick_tile<T, NP, ROWS, 0>(BUDGET);
    static constexpr int LD = 2 * TF + 4;           // row length; columns 2TF+2, 2TF+3: dead writes
    static constexpr int NIT_S = VS * (TF + 1);
    static constexpr int NIT_M = V * (TF + 1);
    static constexpr int ITEMS = ((NIT_S > NIT_M ? NIT_S : NIT_M) + kHalf - 1) / kHalf;
    static constexpr int ROUNDS = ((2 * TF + 1) * NP + kFluxThreads - 1) / kFluxThreads;
    static constexpr int ITEMS3 = (NOUT * TF + kHalf - 1) / kHalf;   // back projection, per side
    static constexpr int LDS_T = ROWS * NP * LD;    // state region (elements of T)
};

struct TileGeom {
    int row, pp, i0, nf;
};

template <typename T>
__device__ __forceinline__ TileGeom tile_geom(const FluxArgs<T> &a, int t, int NP)
{
    TileGeom g;
    const int chunk = t % a.tiles_per_row;
    const int rest = t / a.tiles_per_row;
    g.pp = rest % NP;                       // line p_perp
    g.row = rest / NP;                      // i_perp
    g.i0 = chunk * a.tile_len;
    g.nf = min(a.tile_len, a.n_par - g.i0);
    return g;
}

// Phase 0, in two steps: the face columns of the items this thread projects, then the
// loads of their face lines.  Every lane issues every load (clamped to a valid address,
// the item marked dead) so that the number of vector-memory operations between a load
// and its use is the same on every path: vector-memory operations complete in issue
// order, and the compiler can then wait for exactly the operation it needs instead of
// for all outstanding ones (a lookup issued after the previous tile's stores would
// otherwise also wait for those stores).  The columns of a tile are looked up two tiles
// ahead of its loads.  A column of a dead item (past the tile, or no tile at all) is
// still a valid column; the item is recognised from the geometry where it is used (a
// select on the loaded value here would let the compiler sink the load into a branch).
template <typename C, typename T, int NP>
__device__ __forceinline__ void prefetch_cols(const FluxArgs<T> &a, const TileGeom &g, int side, int lt,
                                              int (&cols)[C::ITEMS])
{
    constexpr int TF = C::TF;
    const int np_ = a.n_par;
    const int32_t *fid = (side ? a.fid_m : a.fid_s) + (size_t)g.row * np_;
    // static slot f: face i0 - 1 + f (slot 0 = halo); moving slot f: face i0 + f - n - 1
    const int off = side ? -a.nmod - 1 : -1;
#pragma unroll
    for (int k = 0; k < C::ITEMS; ++k) {
        const int it = lt + k * kHalf;
        const int v = it / (TF + 1);
        const int f = it - v * (TF + 1);
        int i = g.i0 + min(f, g.nf) + off;
        if (i < 0) i += np_;
        cols[k] = fid[i];
    }
}

template <typename C, typename T, int NP>
__device__ __forceinline__ void prefetch(const FluxArgs<T> &a, const TileGeom &g, int side, int lt,
                                         const int (&cols)[C::ITEMS], T (&u)[C::ITEMS][NP])
{
    constexpr int V = C::V, VS = C::VS, TF = C::TF;
    const size_t plane_s = (size_t)NP * NP * a.nfs, plane_m = (size_t)NP * NP * a.nfm;
    const size_t stride = side ? a.nfm : a.nfs;
#pragma unroll
    for (int k = 0; k < C::ITEMS; ++k) {
        const int it = lt + k * kHalf;
        const int v = min(it / (TF + 1), side ? V - 1 : VS - 1);
        const int c = cols[k];                      // dead items read a valid column
        const T *src = !side ? (v < 5 ? a.Us + v * plane_s
                                      : (v < V ? a.Gs + (v - 5) * plane_s : a.met + (v - V) * plane_s))
                             : (v < 5 ? a.Um + v * plane_m : a.Gm + (v - 5) * plane_m);
        src += c + (size_t)NP * g.pp * stride;
#pragma unroll
        for (int j = 0; j < NP; ++j) u[k][j] = src[(size_t)j * stride];
    }
}

// Output face columns of this thread's back-projection items (item e = lt + k*128 of its
// side: variable e / TF, face f = e % TF of the tile); unconditional loads, as above.
template <typename C, typename T>
__device__ __forceinline__ void out_cols(const FluxArgs<T> &a, const TileGeom &g, int side, int lt,
                                         int (&col3)[C::ITEMS3])
{
    constexpr int TF = C::TF;
    const int np_ = a.n_par;
    const int32_t *fid = (side ? a.fid_m : a.fid_s) + (size_t)g.row * np_;
    const int off = side ? -a.nmod - 1 : 0;   // moving face i0+f-n-1, static face i0+f
#pragma unroll
    for (int k = 0; k < C::ITEMS3; ++k) {
        const int e = lt + k * kHalf;
        const int f = e - (e / TF) * TF;
        int i = g.i0 + min(f, g.nf - 1) + off;
        if (i < 0) i += np_;
        col3[k] = fid[i];
    }
}

// Phase 2 of a tile, shared by the VALU- and the matrix-core-projection kernels: thread
// <-> mortar node (all ROUNDS rounds of 256 points), all variables of both sides from
// LDS (static slot ms at column ms + 1, moving slot ms at column ms, rows of LD), the
// pointwise Riemann + BR1 flux times the surface element, written over the static
// region as fluxes [5][NP][LD] (slot ms at column ms).  Starts after and ends with a
// barrier.
template <typename T, int NP, bool NSV, bool MET, int RIEM, int LD, int ROUNDS>
__device__ __forceinline__ void flux_points(const FluxArgs<T> &a, int nf, const T *ldsS, const T *ldsM,
                                            T *ldsF)
{
    constexpr int V = NSV ? 20 : 5;
    const int tid = threadIdx.x;
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
                unit_normal(nx, ny, nz);
            }
            T F[5];
            Side<T> SL, SR;
            side_state(UL, nx, ny, nz, a.gas, SL);
            side_state(UR, nx, ny, nz, a.gas, SR);
            convective_flux_sides<T, RIEM>(SL, SR, UL, UR, nx, ny, nz, a.gas, F);
            if (NSV) {
                // the viscous fluxes reuse the sides' 1/rho, velocities and pressures
                T G[15], FvL[5], FvR[5];
#pragma unroll
                for (int gg = 0; gg < 15; ++gg) G[gg] = ldsS[((5 + gg) * NP + q) * LD + ms + 1];
                viscous_flux_side(SL, G, nx, ny, nz, a.gas, FvL);
#pragma unroll
                for (int gg = 0; gg < 15; ++gg) G[gg] = ldsM[((5 + gg) * NP + q) * LD + ms];
                viscous_flux_side(SR, G, nx, ny, nz, a.gas, FvR);
#pragma unroll
                for (int v = 0; v < 5; ++v) F[v] -= T(0.5) * (FvL[v] + FvR[v]);
            }
#pragma unroll
            for (int v = 0; v < 5; ++v) res[r][v] = F[v] * dS;
        }
    }
    __syncthreads();   // the flux region overwrites static values still being read
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
}

// Phase 2 of a lifting tile: thread <-> mortar node, the BR1 average of both sides'
// states times each component of the static normal and the surface element (Sec. 2:
// the gradients of the first Bassi-Rebay method lift the interface average of U), 15
// values per node written over the state region as [3][5][NP][LD] (component d,
// variable v at row 5 d + v, slot ms at column ms).  Starts after and ends with a barrier.
template <typename T, int NP, bool MET, int LD, int ROUNDS>
__device__ __forceinline__ void lift_points(const FluxArgs<T> &a, int nf, const T *ldsS, const T *ldsM,
                                            T *ldsF)
{
    const int tid = threadIdx.x;
    const int nm = 2 * nf + 1;
    const int npts = nm * NP;
    T res[ROUNDS][15];
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
        const int pt = tid + r * kFluxThreads;
        if (pt < npts) {
            const int q = pt / nm;
            const int ms = pt - q * nm;
            T n[3] = {a.nx, a.ny, a.nz}, dS = a.dS;
            if (MET) {
#pragma unroll
                for (int d = 0; d < 3; ++d) n[d] = ldsS[((5 + d) * NP + q) * LD + ms + 1];
                dS = ldsS[(8 * NP + q) * LD + ms + 1];
                unit_normal(n[0], n[1], n[2]);
            }
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                const T avg = T(0.5) * (ldsS[(v * NP + q) * LD + ms + 1] + ldsM[(v * NP + q) * LD + ms]) * dS;
#pragma unroll
                for (int d = 0; d < 3; ++d) res[r][5 * d + v] = avg * n[d];
            }
        }
    }
    __syncthreads();   // the output region overwrites states still being read
#pragma unroll
    for (int r = 0; r < ROUNDS; ++r) {
        const int pt = tid + r * kFluxThreads;
        if (pt < npts) {
            const int q = pt / nm;
            const int ms = pt - q * nm;
#pragma unroll
            for (int o = 0; o < 15; ++o) ldsF[(o * NP + q) * LD + ms] = res[r][o];
        }
    }
    __syncthreads();
}

// LDS bytes of one instantiation (state region + matrices).
template <typename T, int NP, bool NSV, bool MET, int BUDGET, bool LIFT = false>
constexpr size_t flux_smem_bytes()
{
    using C = FluxCfg<T, NP, NSV, MET, BUDGET, LIFT>;
    return ((size_t)C::LDS_T * sizeof(T) + 15) / 16 * 16 + (size_t)8 * C::NN * sizeof(T);
}

// All tiles of one interface that this workgroup's cursor visits (the cursor is valid
// on entry).  smem holds flux_smem_bytes() bytes, 16-aligned.  Ends with a barrier, so
// the caller may reuse smem at once.
template <typename T, int NP, bool NSV, bool MET, int RIEM, int BUDGET, bool CONS = true, bool LIFT = false>
__device__ __forceinline__ void run_interface(const FluxArgs<T> &a, TileCursor &cur, char *smem)
{
    using C = FluxCfg<T, NP, NSV, MET, BUDGET, LIFT>;
    constexpr int NOUT = C::NOUT;
    constexpr int V = C::V, VS = C::VS, NN = C::NN, TF = C::TF, LD = C::LD, P = NN;
    static_assert(C::LDS_T * sizeof(T) >= assemble_scratch<NP>() * sizeof(double), "assembly scratch");

    T *lds = reinterpret_cast<T *>(smem);
    T *mats = reinterpret_cast<T *>(smem + ((size_t)C::LDS_T * sizeof(T) + 15) / 16 * 16);
    T *ldsS = lds;                          // static values [VS][NP][LD], slot ms at column ms+1
    T *ldsM = lds + VS * NP * LD;           // moving values [V][NP][LD],  slot ms at column ms
    T *ldsF = lds;                          // fluxes [5][NP][LD] (reuses the static region)

    const int tid = threadIdx.x;
    // 0: static, 1: moving (phases 0, 1, 3); uniform over each wave
    const int side = __builtin_amdgcn_readfirstlane(tid >= kHalf ? 1 : 0);
    const int lt = tid - side * kHalf;
    const int np_ = a.n_par;
    const int nmod = a.nmod;
    const size_t plane_s = (size_t)P * a.nfs, plane_m = (size_t)P * a.nfm;

    // conservation sums of this thread's back-projection items (item k3 always has the
    // same variable), over all its tiles
    // (a plain sum: a thread adds one value per tile)
    double csum[C::ITEMS3], cmag[C::ITEMS3];
#pragma unroll
    for (int k = 0; k < C::ITEMS3; ++k) csum[k] = cmag[k] = 0.0;

    // Pipeline: the face lines of tile t+1 are loaded while tile t is processed; at the
    // start of tile t the input columns of tile t+2 and the output columns of tile t+1
    // are looked up, so every column is in registers before the loads that retire it are
    // waited for.
    const buf_rsrc_t rF = side ? buf_rsrc(a.Fm, (uint32_t)(NOUT * plane_m * sizeof(T)))
                               : buf_rsrc(a.Fs, (uint32_t)(NOUT * plane_s * sizeof(T)));
    const uint32_t nfo = side ? a.nfm : a.nfs;
    TileGeom g = tile_geom(a, cur.tile(), NP);
    cur.next();
    bool more = cur.valid();
    TileGeom gn = tile_geom(a, more ? cur.tile() : 0, NP);
    T u[C::ITEMS][NP];
    int cols[C::ITEMS], cols_n[C::ITEMS], col3[C::ITEMS3], col3_n[C::ITEMS3];
    prefetch_cols<C, T, NP>(a, g, side, lt, cols);
    out_cols<C, T>(a, g, side, lt, col3);
    prefetch_cols<C, T, NP>(a, gn, side, lt, cols_n);
    prefetch<C, T, NP>(a, g, side, lt, cols, u);
    // Stores that write nothing, in the place of the previous tile's: the loop is then
    // entered with the same sequence of outstanding memory operations as it is repeated
    // with, and the compiler's wait for a tile's loads need not also cover the previous
    // tile's stores.
#pragma unroll
    for (int k = 0; k < C::ITEMS3 * NP; ++k)   // distinct offsets: no store is merged away
        buf_store<T>(T(0), rF, kBufOff + (uint32_t)(k * sizeof(T)), 0);

    // FP64 matrices for this stage, once per workgroup and interface
    assemble_matrices<NP, T>(a.basis, a.s, reinterpret_cast<double *>(lds), nullptr, nullptr,
                             mats, mats + 4 * NN);

    while (true) {
        cur.next();
        const bool more2 = cur.valid();
        const TileGeom gnn = tile_geom(a, more2 ? cur.tile() : 0, NP);
        prefetch_cols<C, T, NP>(a, gnn, side, lt, cols);
        out_cols<C, T>(a, gn, side, lt, col3_n);
        // ---- phase 1: forward projection (register mat-vec) ------------------------
        {
            // static: Pf0 -> slot 2f-1 (column 2f), Pf1 -> slot 2f (column 2f+1)
            // moving: Pf3 (lower part) -> slot 2f (column 2f), Pf2 (upper) -> slot 2f+1
            // Every item is projected (no branch, so each matrix row is read once for all
            // of this thread's items) and written as one pair (columns 2f, 2f+1): the
            // static column 0 and the columns of faces past the tile are never read, and
            // items past the last variable write the two spare columns of the last one.
            const T *PA = mats + (side ? 3 : 0) * NN;
            const T *PB = mats + (side ? 2 : 1) * NN;
            T *base = side ? ldsM : ldsS;
            const int nit = side ? C::NIT_M : C::NIT_S;
            const int vlast = side ? V - 1 : VS - 1;
            int woff[C::ITEMS];
#pragma unroll
            for (int k = 0; k < C::ITEMS; ++k) {
                const int it = lt + k * kHalf;
                const int v = it / (TF + 1);
                const int f = it - v * (TF + 1);
                woff[k] = it < nit ? v * NP * LD + 2 * f : vlast * NP * LD + 2 * TF + 2;
            }
            typedef T T2 __attribute__((ext_vector_type(2)));
#pragma unroll
            for (int q = 0; q < NP; ++q) {
                T pa[NP], pb[NP];
#pragma unroll
                for (int j = 0; j < NP; ++j) {
                    pa[j] = PA[q * NP + j];
                    pb[j] = PB[q * NP + j];
                }
#pragma unroll
                for (int k = 0; k < C::ITEMS; ++k) {
                    T qa = T(0), qb = T(0);
#pragma unroll
                    for (int j = 0; j < NP; ++j) {
                        qa += pa[j] * u[k][j];
                        qb += pb[j] * u[k][j];
                    }
                    *reinterpret_cast<T2 *>(base + woff[k] + q * LD) = T2{qa, qb};
                }
            }
        }
        // the next tile's loads fly while this tile's flux and back projection run (dead
        // loads after the last tile)
        prefetch<C, T, NP>(a, gn, side, lt, cols_n, u);
        __syncthreads();

        // ---- phase 2: flux at every mortar node -------------------------------------
        if constexpr (LIFT) lift_points<T, NP, MET, LD, C::ROUNDS>(a, g.nf, ldsS, ldsM, ldsF);
        else flux_points<T, NP, NSV, MET, RIEM, LD, C::ROUNDS>(a, g.nf, ldsS, ldsM, ldsF);

        // ---- phase 3: back projection, threads 0-127 static, 128-255 moving ----------
        // static face i0+f: mortars (i0+f, 0) slot 2f+1 and (i0+f, 1) slot 2f+2
        // moving face i0+f-n-1: lower (i0+f-1, 1) slot 2f, upper (i0+f, 0) slot 2f+1
        {
            const T *B_lo = mats + 4 * NN + (side ? 3 : 0) * NN;
            const T *B_hi = mats + 4 * NN + (side ? 2 : 1) * NN;
#pragma unroll
            for (int k3 = 0; k3 < C::ITEMS3; ++k3) {
                // the matrices are read again for every item: kept in registers across
                // items they would take 2 NP^2 of them
                asm volatile("" ::: "memory");
                const int e = lt + k3 * kHalf;
                const int ve = e / TF;
                const int f = e - ve * TF;
                const int v = min(ve, NOUT - 1);
                const T *src = ldsF + v * NP * LD;
                const int s0 = side ? 2 * f : 2 * f + 1;
                T lo[NP], hi[NP];
#pragma unroll
                for (int q = 0; q < NP; ++q) {
                    lo[q] = src[q * LD + s0];
                    hi[q] = src[q * LD + s0 + 1];
                }
                // every lane stores; a dead item's offset lies beyond the array
                const bool ok = e < NOUT * TF && f < g.nf;
                const uint32_t o0 = ((uint32_t)(v * NN + NP * g.pp) * nfo + (uint32_t)col3[k3]) * (uint32_t)sizeof(T);
                double ls = 0.0, lm = 0.0;       // this face line's w_j-weighted sums
#pragma unroll
                for (int j = 0; j < NP; ++j) {
                    T acc = T(0);
#pragma unroll
                    for (int q = 0; q < NP; ++q) {
                        acc += B_lo[j * NP + q] * lo[q];   // contracted to one FMA each
                        acc += B_hi[j * NP + q] * hi[q];
                    }
                    buf_store<T>(acc, rF, ok ? o0 + (uint32_t)(j * sizeof(T)) * nfo : kBufOff, 0);
                    const double y = a.basis->w[j] * (double)acc;
                    ls += y;
                    lm += fabs(y);
                }
                if (CONS && !LIFT && a.cons && ok) {
                    const double wl = a.basis->w[g.pp];
                    csum[k3] += wl * ls;
                    cmag[k3] += wl * lm;
                }
            }
        }
        __syncthreads();   // phase 3 reads the LDS that the next phase 1 overwrites
        if (!more) break;
        g = gn;
        gn = gnn;
        more = more2;
#pragma unroll
        for (int k = 0; k < C::ITEMS; ++k) cols_n[k] = cols[k];
#pragma unroll
        for (int k = 0; k < C::ITEMS3; ++k) col3[k] = col3_n[k];
    }

    // conservation partials: per (variable, side) group, one side at a time, thread v
    // adds the side's items e = v TF .. v TF + TF - 1 (thread e % 128, item e / 128) in a
    // fixed order
    if constexpr (CONS && !LIFT) {
        static_assert(C::LDS_T * sizeof(T) >= (size_t)kHalf * C::ITEMS3 * 2 * sizeof(double),
                      "conservation staging");
        if (a.cons) {
            double *red = reinterpret_cast<double *>(smem);
            for (int sd = 0; sd < 2; ++sd) {
                if (side == sd) {
#pragma unroll
                    for (int k = 0; k < C::ITEMS3; ++k) {
                        red[(lt * C::ITEMS3 + k) * 2 + 0] = csum[k];
                        red[(lt * C::ITEMS3 + k) * 2 + 1] = cmag[k];
                    }
                }
                __syncthreads();
                if (tid < 5) {
                    ConsSum t;
                    double m = 0.0;
                    for (int e = tid * TF; e < (tid + 1) * TF; ++e) {
                        const double *r = red + ((e % kHalf) * C::ITEMS3 + e / kHalf) * 2;
                        t.add(r[0]);
                        m += r[1];
                    }
                    const size_t o = ((size_t)(2 * tid + sd) * gridDim.x + blockIdx.x) * 2;
                    a.cons[o + 0] = t.value();
                    a.cons[o + 1] = m;
                }
                __syncthreads();
            }
        }
    }
}

template <typename T, int NP, bool NSV, bool MET, int RIEM, int BUDGET>
__global__ __launch_bounds__(kFluxThreads) void k_mortar_flux(FluxArgs<T> a)
{
    __shared__ __attribute__((aligned(16))) char smem[flux_smem_bytes<T, NP, NSV, MET, BUDGET>()];
    TileCursor cur(a.n_tiles);
    if (!cur.valid()) {                     // uniform over the workgroup
        cons_zero(a.cons);
        return;
    }
    run_interface<T, NP, NSV, MET, RIEM, BUDGET>(a, cur, smem);
}

// The BR1 lifting surface term of one interface (a.Fs / a.Fm: [3][5][P][n_face] outputs;
// a.Gs / a.Gm unused).
template <typename T, int NP, bool MET, int BUDGET>
__global__ __launch_bounds__(kFluxThreads) void k_mortar_lift(FluxArgs<T> a)
{
    __shared__ __attribute__((aligned(16))) char smem[flux_smem_bytes<T, NP, false, MET, BUDGET, true>()];
    TileCursor cur(a.n_tiles);
    if (!cur.valid()) return;               // uniform over the workgroup
    run_interface<T, NP, false, MET, 0, BUDGET, false, true>(a, cur, smem);
}

// ---- several interfaces in one persistent launch ---------------------------------------

constexpr int kMaxBatch = 8;

template <typename T>
struct BatchArgs {
    FluxArgs<T> a[kMaxBatch];        // a[i].n_tiles: tiles of interface i
    int np[kMaxBatch];
    int met[kMaxBatch];
    int n_if;
};

template <int MASK>
constexpr int mask_max_np()
{
    int m = 0;
    for (int np = 2; np <= kMaxNP; ++np)
        if (MASK & (1 << np)) m = np;
    return m;
}

template <typename T, bool NSV, int BUDGET, int NP>
constexpr size_t pair_smem()
{
    return flux_smem_bytes<T, NP, NSV, false, BUDGET>() > flux_smem_bytes<T, NP, NSV, true, BUDGET>()
               ? flux_smem_bytes<T, NP, NSV, false, BUDGET>()
               : flux_smem_bytes<T, NP, NSV, true, BUDGET>();
}

template <typename T, bool NSV, int BUDGET, int MASK>
constexpr size_t batch_smem()
{
    size_t m = 0;
#define MORTAR_SMEM_NP(NPV) \
    if ((MASK & (1 << NPV)) && pair_smem<T, NSV, BUDGET, NPV>() > m) m = pair_smem<T, NSV, BUDGET, NPV>();
    MORTAR_SMEM_NP(2) MORTAR_SMEM_NP(3) MORTAR_SMEM_NP(4) MORTAR_SMEM_NP(5) MORTAR_SMEM_NP(6)
    MORTAR_SMEM_NP(7) MORTAR_SMEM_NP(8) MORTAR_SMEM_NP(9) MORTAR_SMEM_NP(10)
#undef MORTAR_SMEM_NP
    return m;
}

// The workgroups take the interfaces one after the other; for each, every XCD gets the
// same share of its tiles (see TileCursor) and each workgroup assembles that interface's
// matrices once.  MASK: bit NP set for every degree this instantiation serves; the host
// only launches it for batches whose degrees are all in MASK.
// One interface of a batch as a real call: each degree's code keeps its own register
// allocation, so the batched kernel needs only as many registers as its largest
// degree (inlining every degree into one body costs more than any of them alone).
template <typename T, int NP, bool NSV, bool MET, int RIEM, int BUDGET>
__device__ __noinline__ void run_interface_call(const FluxArgs<T> *a, char *smem)
{
    TileCursor cur(a->n_tiles);
    run_interface<T, NP, NSV, MET, RIEM, BUDGET, false>(*a, cur, smem);
}

template <typename T, int NP, bool NSV, bool MET, int RIEM, int BUDGET, bool CALL>
__device__ __forceinline__ void run_batch_member(const FluxArgs<T> *a, char *smem)
{
    if constexpr (CALL) {
        run_interface_call<T, NP, NSV, MET, RIEM, BUDGET>(a, smem);
    } else {
        TileCursor cur(a->n_tiles);
        run_interface<T, NP, NSV, MET, RIEM, BUDGET, false>(*a, cur, smem);
    }
}

// The three-degree turbine set is inlined with the register budget of two waves per
// SIMD; the every-degree instantiation calls one function per degree.
template <int MASK>
constexpr bool batch_calls() { return MASK != kMaskTurbine; }

template <typename T, bool NSV, int RIEM, int BUDGET, int MASK>
__global__ __launch_bounds__(kFluxThreads) __attribute__((amdgpu_waves_per_eu(2)))
void k_mortar_flux_batch(BatchArgs<T> b)
{
    __shared__ __attribute__((aligned(16))) char smem[batch_smem<T, NSV, BUDGET, MASK>()];
    constexpr bool CALL = batch_calls<MASK>();
    for (int i = 0; i < b.n_if; ++i) {
        if (!TileCursor(b.a[i].n_tiles).valid()) continue;   // uniform over the workgroup
        const bool met = b.met[i] != 0;
#define MORTAR_BATCH_NP(NPV)                                                             \
    if ((MASK & (1 << NPV)) && b.np[i] == NPV) {                                         \
        if (met) run_batch_member<T, NPV, NSV, true, RIEM, BUDGET, CALL>(&b.a[i], smem); \
        else run_batch_member<T, NPV, NSV, false, RIEM, BUDGET, CALL>(&b.a[i], smem);    \
        continue;                                                                        \
    }
        MORTAR_BATCH_NP(2) MORTAR_BATCH_NP(3) MORTAR_BATCH_NP(4) MORTAR_BATCH_NP(5)
        MORTAR_BATCH_NP(6) MORTAR_BATCH_NP(7) MORTAR_BATCH_NP(8) MORTAR_BATCH_NP(9)
        MORTAR_BATCH_NP(10)
#undef MORTAR_BATCH_NP
    }
}

}  // namespace mortar
