// Internal declarations of the MI355X mortar library (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>
#include <vector>

#include "mortar.h"

namespace mortar {

constexpr int kMaxN = 15;
constexpr int kMaxNP = kMaxN + 1;
// Degrees up to kMaxNFast (NP <= 10) have every kernel variant, batching and the bf16/fp16
// modes; higher degrees run the VALU-projection kernel, one launch per interface.
constexpr int kMaxNFast = 9;
constexpr int kMaxOwners = 1024;   // distinct owner ranks per side (index-map sort keys)
constexpr int kSortBlock = 256;    // elements per block of the index-map counting sort

// Static-to-moving pairing (Sec. 4.3, index relation): mortar (i_par, i_sub) of a row lies
// on the moving face (i_par - n + i_sub - 1) mod n_par of the same row; nmod = n mod
// n_par in [0, n_par).  0-based indices, periodic wrap along the slide.
__host__ __device__ inline int moving_partner(int i_par, int i_sub, int nmod, int n_par)
{
    int j = (i_par - nmod + i_sub - 1) % n_par;   // in (-n_par, n_par)
    return j < 0 ? j + n_par : j;
}

// Run-time NP -> compile-time instantiation: f(std::integral_constant<int, NP>) for NP in
// [LO, HI], dflt otherwise.
template <int LO, int HI, typename R, typename F>
inline R np_dispatch(int NP, R dflt, F &&f)
{
    if constexpr (LO > HI) {
        (void)NP;
        (void)f;
        return dflt;
    } else {
        if (NP == LO) return f(std::integral_constant<int, LO>{});
        return np_dispatch<LO + 1, HI, R>(NP, dflt, f);
    }
}

// Per-interface device parameter block, rewritten by the assembly kernel every stage.
// Header followed by matrices: double Pf[4][NP][NP], double Pb[4][NP][NP],
// float Pf[4][NP][NP], float Pb[4][NP][NP].  Matrix order k: static i_sub 0, static
// i_sub 1, moving i_sub 0 (upper part of the moving face), moving i_sub 1 (lower part).
struct alignas(16) ParamHeader {
    int32_t nmod;  // n mod n_par
    int32_t NP;
    int64_t n;
    double s;
    double pad;
};
constexpr size_t kHeaderBytes = sizeof(ParamHeader);  // 32

__host__ __device__ inline size_t param_bytes(int NP) {
    // 8 matrices (4 forward, 4 backward) in double and again in float
    return kHeaderBytes + (size_t)8 * NP * NP * (sizeof(double) + sizeof(float));
}
__host__ __device__ inline size_t off_f64(int) { return kHeaderBytes; }
__host__ __device__ inline size_t off_f32(int NP) { return kHeaderBytes + (size_t)8 * NP * NP * sizeof(double); }

// FP64 constants of one interface's basis, uploaded once at setup (Sec. 3.2: the mass
// matrix depends only on the basis).
struct BasisConsts {
    double x[kMaxNP];                 // nodes
    double w[kMaxNP];                 // quadrature weights of the nodes
    double bw[kMaxNP];                // barycentric weights 1 / prod_{m != j} (x_j - x_m)
    double t[kMaxNP];                 // Gauss rule used for S (exact for degree 2N)
    double tw[kMaxNP];
    double Lt[kMaxNP * kMaxNP];       // l_q(t_r), [r][q]
    double Minv[kMaxNP * kMaxNP];     // inverse mass matrix
};

struct Iface {
    mortar_iface_desc d{};
    int NP = 0, P = 0, F = 0;          // points per direction, per face, face pairs
    size_t elem = 8;                   // bytes per element of U/G/F
    // device buffers
    int32_t *d_fid_s = nullptr, *d_fid_m = nullptr;
    int32_t *d_oid_s = nullptr, *d_oid_m = nullptr;  // dense owner ids [n_perp*n_par]
    int32_t *d_oval_s = nullptr, *d_oval_m = nullptr; // owner value per dense id
    int R_s = 1, R_m = 1;              // distinct owners per side
    void *d_metrics = nullptr;         // [4][P][n_face_static] in element type, or null
    char *d_params = nullptr;          // ParamHeader + matrices
    BasisConsts *d_basis = nullptr;
    int32_t *d_A[2] = {nullptr, nullptr};  // [5][2F] per side
    int32_t *d_m[2] = {nullptr, nullptr};  // [2][n_face] per side
    int32_t *d_hist = nullptr;             // [R][n_sort_blocks] counting-sort scratch
    int32_t *d_pair = nullptr;             // [2][n_par] pairing, written by mortar_get_pairing
    int n_sort_blocks = 0;
    int64_t n = 0;
    double s = 0.0;
    int64_t nmod_built = -1;           // n mod n_par of the current index map
    bool ready = false;
    double *d_cons = nullptr;          // conservation partials [10][blocks][4]
    double *d_cons_wg = nullptr;       // partials of the fused flux launch [10][kConsGridMax][2]
    // the flux launch whose fused partials d_cons_wg holds: output arrays and grid (0: none)
    mutable const void *cons_Fs = nullptr, *cons_Fm = nullptr;
    mutable int cons_nb = 0;
    double *d_cons_out = nullptr;      // conservation sums [5][3] of the last host query
    int n_cons_blocks = 0;
    int flux_occ = 1;                  // resident flux workgroups per CU
    int flux_variant = 0;              // 0: VALU projections, 1: matrix-core projections
                                       // staged in LDS, 2: register-direct matrix-core kernel
    int lp = 0;                        // GEMM operands: 0 element type, 1 bf16, 2 fp16
    int tune_tile = 0;                 // tile length cap from tuning (0: variant's largest)
    int tune_grid = 0;                 // workgroups from tuning (0: all resident slots)
};

struct Handle {
    int device = 0;
    int n_cu = 256;
    bool batched = false;              // all interfaces go in one persistent launch
    bool batch_turbine = false;        // the N = 3, 5, 7 instantiation covers the batch
    int batch_occ = 1;
    int tune_grid_batch = 0;           // workgroups of the batched launch (0: default)
    int batch_variant = 0;             // batched kernel: 0 VALU projections, 2 register-direct
    bool batch_rd_ok = false;          // the register-direct batch kernel covers the batch
    int batch_occ_rd = 1;
    unsigned tune_epoch = 0;           // bumped by every tuning change
    double *static_scratch = nullptr;  // this device's address of the static partials array
    std::vector<Iface> ifs;
};

// ---- launchers (kernels in k_*.hip) ------------------------------------------------
hipError_t launch_assemble(const Iface &f, hipStream_t st);
hipError_t launch_index_map(Iface &f, int side, hipStream_t st);
hipError_t launch_pairing(const Iface &f, hipStream_t st);
hipError_t launch_flux(const Iface &f, int n_cu, const void *Us, const void *Um, const void *Gs,
                       const void *Gm, void *Fs, void *Fm, hipStream_t st);
struct Handle;
hipError_t launch_flux_batched(const Handle &h, const void *const *Us, const void *const *Um,
                               const void *const *Gs, const void *const *Gm, void *const *Fs,
                               void *const *Fm, hipStream_t st);
int cons_blocks(int P, int nfaces);
// Largest flux grid whose workgroups write conservation partials.
constexpr int kConsGridMax = 4096;
// Waves of a register-direct workgroup; they take consecutive tiles of one line.  In the
// lockstep launches (4-byte data: Navier-Stokes, and Euler from kRdLockEulerNP nodes per
// line on) they go through the rounds of tiles together (a workgroup barrier per round),
// so the cache lines that neighbouring tiles share (a tile's 16 face slots span 64 bytes
// of each 128-byte line of a (variable, node) row, and consecutive tiles overlap by the
// halo face) are requested by several waves of one CU at about the same time: fetched
// from HBM once, and written back once when their two halves come from two tiles.  Eight
// waves (two per SIMD, the occupancy of those launches).  The other launches run four
// independent waves per workgroup (the finer granularity keeps their higher occupancy,
// three or four waves per SIMD, which an eight-wave workgroup with its 80 KB of
// conservation slots would lose).
constexpr int kRdLockWaves = 8;
// The lockstep waves go in two groups out of phase: waves WV/2.. meet at the top of a
// round, waves 0..WV/2-1 after issuing the round's loads.  A barrier then releases the
// first group into its wait for the loads it has just issued while the second group
// issues its own, and the first group issues the next round's loads as soon as its
// arithmetic is done, while the second group still computes: each group's load latency
// overlaps the other group's arithmetic on the same CU, where one barrier for all would
// have every wave of the CU wait for memory at once.
constexpr bool kRdPingPong = true;
// The two groups take tiles from the two halves of each XCD's share (HalfCursor).
constexpr bool kRdSplitHalves = true;
// Euler launches with 4-byte data run in lockstep from this many nodes per line on (N = 7:
// two waves per SIMD already; plane N = 9 Euler: 253 -> 223 us in FP32, reads 1.14x ->
// 1.01x and writes 1.35x -> 1.02x the algorithmic bytes).
constexpr int kRdLockEulerNP = 8;
__host__ __device__ constexpr bool rd_lockstep(int elem_bytes, bool ns, int np)
{
    return elem_bytes == 4 && (ns || np >= kRdLockEulerNP);
}
__host__ __device__ constexpr int rd_waves(int elem_bytes, bool ns, int np)
{
    return rd_lockstep(elem_bytes, ns, np) ? kRdLockWaves : 4;
}
// The register-direct lifting launches (FP32): lockstep rounds of eight waves from this
// many nodes per line on (two waves per SIMD there; the rounds write each line's two
// halves together: annulus N = 7 lifting 165 -> 111.5 us), four free waves below.
constexpr int kRdLockLiftNP = 8;
__host__ __device__ constexpr int rd_lift_waves(int np) { return np >= kRdLockLiftNP ? kRdLockWaves : 4; }
// the batch kernel (4-byte data, both physics)
constexpr int kRdBatchWaves = kRdLockWaves;
// Largest array (bytes) the register-direct kernels address with 32-bit buffer offsets;
// offsets from there up to 4 GiB mark masked-off lanes.
constexpr int64_t kRdMaxBytes = 0xFFFFFF00;
// Output faces per tile of the register-direct kernels (16 slots, one is the halo).
constexpr int kRdTileFaces = 15;
hipError_t launch_conservation_final(const Iface &f, double *d_out, hipStream_t st);
constexpr int kMaxConsBatch = 8;
hipError_t launch_conservation_final_batch(const Iface *const *fs, double *const *outs, int n,
                                           hipStream_t st);
// Conservation sums with the partials in the library's static device array: at most
// kStaticConsIfaces interfaces per call, one slot of kStaticConsSlot doubles each (10
// groups x the conservation grid's at most 1024 blocks x 2).
constexpr int kStaticConsIfaces = 8;
constexpr int kStaticConsSlot = 10 * 1024 * 2;
constexpr int kMaxDevices = 64;
hipError_t static_cons_scratch(int device, double **out);
hipError_t launch_conservation_static(const Iface &f, int slot, double *scratch_ptr,
                                      const void *Fs, const void *Fm, double *d_out, hipStream_t st);
hipError_t launch_conservation(const Iface &f, const void *Fs, const void *Fm, double *d_out,
                               hipStream_t st);

}  // namespace mortar
