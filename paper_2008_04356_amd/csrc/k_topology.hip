// Per-stage topology kernels of the mortar operator:
//  - FP64 projection matrices of the current s for inspection (the flux kernel
//    assembles its own copy in its prologue with the same routine);
//  - the device-side mortar sort (Sec. 4.4, Appendix A): sorted index array A and its
//    inverse map m, rebuilt when the displacement crosses a whole face;
//  - FP64 compensated conservation sums of the face fluxes of both sides.
#include <algorithm>

#include "assemble.h"
#include "mortar_internal.h"

namespace mortar {

// ------------------------------------------------------------------------------------
// Projection matrices for inspection: the same device routine the flux kernel runs in
// its prologue, written to the handle's FP64 buffer.
// ------------------------------------------------------------------------------------

template <int NP>
__global__ void k_assemble_inspect(const BasisConsts *__restrict__ basis, double s,
                                   char *__restrict__ params)
{
    __shared__ double work[8 * NP * NP];
    double *Pf = reinterpret_cast<double *>(params + kHeaderBytes);
    assemble_matrices<NP, double>(basis, s, work, Pf, Pf + 4 * NP * NP, (double *)nullptr,
                                  (double *)nullptr);
}

hipError_t launch_assemble(const Iface &f, hipStream_t st)
{
#define MORTAR_ASM_CASE(np)                                                                   \
    case np:                                                                                  \
        hipLaunchKernelGGL(k_assemble_inspect<np>, dim3(1), dim3(128), 0, st, f.d_basis, f.s, \
                           f.d_params);                                                       \
        break;
    switch (f.NP) {
        MORTAR_ASM_CASE(2) MORTAR_ASM_CASE(3) MORTAR_ASM_CASE(4) MORTAR_ASM_CASE(5)
        MORTAR_ASM_CASE(6) MORTAR_ASM_CASE(7) MORTAR_ASM_CASE(8) MORTAR_ASM_CASE(9)
        MORTAR_ASM_CASE(10)
    default: return hipErrorInvalidValue;
    }
#undef MORTAR_ASM_CASE
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// Index map: stable counting sort by owner over the mortars enumerated in
// (i_par, i_perp, i_sub) order, which equals the nested sort by
// (owner, i_par, i_perp, i_sub) because those three keys enumerate every mortar once.
// ------------------------------------------------------------------------------------

struct MapArgs {
    const int32_t *fid;       // this side's face ids [n_perp*n_par]
    const int32_t *oid_opp;   // dense owner ids of the opposite side [n_perp*n_par]
    const int32_t *oval_opp;  // owner value per dense id
    int32_t *hist;            // [R][nblk]
    int32_t *A;               // [5][E]
    int32_t *m;               // [2][n_face]
    int n_par, n_perp, nmod, side, R, E, n_face;
};

// Element e = (i_par * n_perp + i_perp) * 2 + i_sub -> owner id of the opposite face and
// this side's face column.
__device__ static inline void map_element(const MapArgs &a, int e, int &ia, int &ip, int &k,
                                          int &oid, int &col)
{
    k = e & 1;
    const int r = e >> 1;
    ia = r / a.n_perp;
    ip = r - ia * a.n_perp;
    int jt = ia - a.nmod + k - 1;          // moving index of the mortar (index relation)
    jt %= a.n_par;
    if (jt < 0) jt += a.n_par;
    if (a.side == 0) {                     // static side: owner of the moving face
        oid = a.oid_opp[ip * a.n_par + jt];
        col = a.fid[ip * a.n_par + ia];
    } else {                               // moving side: owner of the static face
        oid = a.oid_opp[ip * a.n_par + ia];
        col = a.fid[ip * a.n_par + jt];
    }
}

__global__ void k_map_count(MapArgs a)
{
    __shared__ int cnt[kMaxOwners];
    for (int r = threadIdx.x; r < a.R; r += blockDim.x) cnt[r] = 0;
    __syncthreads();
    const int e = blockIdx.x * kSortBlock + threadIdx.x;
    if (e < a.E) {
        int ia, ip, k, oid, col;
        map_element(a, e, ia, ip, k, oid, col);
        atomicAdd(&cnt[oid], 1);
    }
    __syncthreads();
    const int nblk = gridDim.x;
    for (int r = threadIdx.x; r < a.R; r += blockDim.x) a.hist[r * nblk + blockIdx.x] = cnt[r];
}

// Exclusive scan of hist (owner-major) in one workgroup.
__global__ void k_map_scan(int32_t *hist, int total)
{
    __shared__ int part[1024];
    const int T = blockDim.x;
    const int per = (total + T - 1) / T;
    const int b = threadIdx.x * per, e = min(total, b + per);
    int sum = 0;
    for (int i = b; i < e; ++i) sum += hist[i];
    part[threadIdx.x] = sum;
    __syncthreads();
    if (threadIdx.x == 0) {
        int run = 0;
        for (int t = 0; t < T; ++t) {
            const int v = part[t];
            part[t] = run;
            run += v;
        }
    }
    __syncthreads();
    int run = part[threadIdx.x];
    for (int i = b; i < e; ++i) {
        const int v = hist[i];
        hist[i] = run;
        run += v;
    }
}

__global__ void k_map_fill(int32_t *m, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) m[i] = -1;
}

__global__ void k_map_scatter(MapArgs a)
{
    __shared__ int own[kSortBlock];
    const int e = blockIdx.x * kSortBlock + threadIdx.x;
    int ia = 0, ip = 0, k = 0, oid = -1, col = 0;
    if (e < a.E) map_element(a, e, ia, ip, k, oid, col);
    own[threadIdx.x] = oid;
    __syncthreads();
    if (e >= a.E) return;
    int rank = 0;  // earlier elements of this block with the same owner
    for (int t = 0; t < (int)threadIdx.x; ++t) rank += (own[t] == oid);
    const int im = a.hist[oid * gridDim.x + blockIdx.x] + rank;
    a.A[0 * a.E + im] = a.oval_opp[oid];
    a.A[1 * a.E + im] = ia;
    a.A[2 * a.E + im] = ip;
    a.A[3 * a.E + im] = k;
    a.A[4 * a.E + im] = col;
    a.m[k * a.n_face + col] = im;
}

hipError_t launch_index_map(Iface &f, int side, hipStream_t st)
{
    MapArgs a;
    a.fid = side == 0 ? f.d_fid_s : f.d_fid_m;
    a.oid_opp = side == 0 ? f.d_oid_m : f.d_oid_s;
    a.oval_opp = side == 0 ? f.d_oval_m : f.d_oval_s;
    a.R = side == 0 ? f.R_m : f.R_s;
    a.hist = f.d_hist;
    a.A = f.d_A[side];
    a.m = f.d_m[side];
    a.n_par = f.d.n_par;
    a.n_perp = f.d.n_perp;
    const int64_t np = f.d.n_par;
    a.nmod = (int)(((f.n % np) + np) % np);
    a.side = side;
    a.E = 2 * f.F;
    a.n_face = side == 0 ? f.d.n_face_static : f.d.n_face_moving;
    const int nblk = f.n_sort_blocks;
    hipLaunchKernelGGL(k_map_fill, dim3((2 * a.n_face + 255) / 256), dim3(256), 0, st, a.m,
                       2 * a.n_face);
    hipLaunchKernelGGL(k_map_count, dim3(nblk), dim3(kSortBlock), 0, st, a);
    hipLaunchKernelGGL(k_map_scan, dim3(1), dim3(1024), 0, st, a.hist, a.R * nblk);
    hipLaunchKernelGGL(k_map_scatter, dim3(nblk), dim3(kSortBlock), 0, st, a);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// Conservation sums (FP64, compensated).  Each block sums a fixed set of (point, face)
// elements of both sides for all five variables; the threads of a block and then the
// block partials are combined by fixed LDS trees, so the result is deterministic.  Each
// accumulator is a Neumaier pair (sum, correction).
// ------------------------------------------------------------------------------------

struct Neumaier {
    double s = 0.0, c = 0.0;
    __device__ void add(double x)
    {
        const double t = s + x;
        c += (fabs(s) >= fabs(x)) ? (s - t) + x : (x - t) + s;
        s = t;
    }
    __device__ void merge(double os, double oc)
    {
        add(os);
        c += oc;
    }
};

// Deterministic in-block combination of 256 threads' Neumaier pairs for NV values: a
// fixed halving tree in LDS.  Every thread must call it; the result is in thread 0.
template <int NV>
__device__ void cons_block_tree(Neumaier (&acc)[NV], double (*red)[256][2])
{
    const int t = threadIdx.x;
#pragma unroll
    for (int e = 0; e < NV; ++e) {
        red[e][t][0] = acc[e].s;
        red[e][t][1] = acc[e].c;
    }
    __syncthreads();
    for (int stride = 128; stride > 0; stride >>= 1) {
        if (t < stride) {
#pragma unroll
            for (int e = 0; e < NV; ++e) {
                Neumaier x;
                x.s = red[e][t][0];
                x.c = red[e][t][1];
                x.merge(red[e][t + stride][0], red[e][t + stride][1]);
                red[e][t][0] = x.s;
                red[e][t][1] = x.c;
            }
        }
        __syncthreads();
    }
    if (t == 0) {
#pragma unroll
        for (int e = 0; e < NV; ++e) {
            acc[e].s = red[e][0][0];
            acc[e].c = red[e][0][1];
        }
    }
}

// Block b sums a fixed set of (point, face) elements of both sides for all five
// variables: element k = p * nfaces + f, k = b*256 + t + j*gridDim*256.
template <typename T>
__global__ __launch_bounds__(256) void k_cons_partial(const T *__restrict__ Fs,
                                                      const T *__restrict__ Fm,
                                                      const int32_t *__restrict__ fid_s,
                                                      const int32_t *__restrict__ fid_m,
                                                      const BasisConsts *__restrict__ basis,
                                                      int NP, int nfaces, int nfs, int nfm,
                                                      double *__restrict__ part)
{
    // part[block][v * 3 + sum][2]: sums = static integral, moving integral, sum of |terms|
    __shared__ double red[15][256][2];
    __shared__ double wq[kMaxNP * kMaxNP];
    const int P = NP * NP;
    for (int p = threadIdx.x; p < P; p += blockDim.x) wq[p] = basis->w[p % NP] * basis->w[p / NP];
    __syncthreads();
    Neumaier acc[15];
    const size_t ps = (size_t)P * nfs, pm = (size_t)P * nfm;
    const int64_t total = (int64_t)P * nfaces;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t k0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k0 < total; k0 += 4 * stride) {
        // four elements per pass: their loads are all issued before the first add
        T xs[4][5], ys[4][5];
        double w[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t k = k0 + u * stride;
            const bool ok = k < total;
            const int p = ok ? (int)(k / nfaces) : 0, f = ok ? (int)(k - (int64_t)p * nfaces) : 0;
            w[u] = ok ? wq[p] : 0.0;
            const size_t os = (size_t)p * nfs + fid_s[f], om = (size_t)p * nfm + fid_m[f];
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                xs[u][v] = Fs[v * ps + os];
                ys[u][v] = Fm[v * pm + om];
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 5; ++v) {
                const double x = w[u] * (double)xs[u][v];
                const double y = w[u] * (double)ys[u][v];
                acc[v * 3 + 0].add(x);
                acc[v * 3 + 1].add(y);
                acc[v * 3 + 2].add(fabs(x) + fabs(y));
            }
    }
    cons_block_tree<15>(acc, red);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int e = 0; e < 15; ++e) {
            part[(size_t)blockIdx.x * 30 + e * 2 + 0] = acc[e].s;
            part[(size_t)blockIdx.x * 30 + e * 2 + 1] = acc[e].c;
        }
    }
}

__global__ __launch_bounds__(256) void k_cons_final(const double *__restrict__ part, int nblk,
                                                    double *__restrict__ out)
{
    __shared__ double red[15][256][2];
    Neumaier acc[15];
    for (int b = threadIdx.x; b < nblk; b += blockDim.x)
#pragma unroll
        for (int e = 0; e < 15; ++e) acc[e].merge(part[(size_t)b * 30 + e * 2 + 0], part[(size_t)b * 30 + e * 2 + 1]);
    cons_block_tree<15>(acc, red);
    if (threadIdx.x == 0)
#pragma unroll
        for (int e = 0; e < 15; ++e) out[e] = acc[e].s + acc[e].c;
}

// Blocks of the conservation sums: about four (point, face) elements per thread, at
// most 2048 blocks.
int cons_blocks(int P, int nfaces)
{
    const int64_t total = (int64_t)P * nfaces;
    return (int)std::max<int64_t>(1, std::min<int64_t>(2048, (total + 1023) / 1024));
}

hipError_t launch_conservation(const Iface &f, const void *Fs, const void *Fm, double *d_out,
                               hipStream_t st)
{
    const int nblk = cons_blocks(f.P, f.F);
    const dim3 grid(nblk);
    if (f.d.precision == MORTAR_FP64)
        hipLaunchKernelGGL(k_cons_partial<double>, grid, dim3(256), 0, st,
                           (const double *)Fs, (const double *)Fm, f.d_fid_s, f.d_fid_m,
                           f.d_basis, f.NP, f.F, f.d.n_face_static, f.d.n_face_moving, f.d_cons);
    else
        hipLaunchKernelGGL(k_cons_partial<float>, grid, dim3(256), 0, st,
                           (const float *)Fs, (const float *)Fm, f.d_fid_s, f.d_fid_m,
                           f.d_basis, f.NP, f.F, f.d.n_face_static, f.d.n_face_moving, f.d_cons);
    hipLaunchKernelGGL(k_cons_final, dim3(1), dim3(256), 0, st, f.d_cons, nblk, d_out);
    return hipGetLastError();
}

}  // namespace mortar
