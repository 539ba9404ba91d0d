// Per-stage topology kernels of the mortar operator:
//  - FP64 projection matrices of the current s for inspection (the flux kernel
//    assembles its own copy in its prologue with the same routine);
//  - the device-side mortar sort (Sec. 4.4, Appendix A): sorted index array A and its
//    inverse map m, rebuilt when the displacement crosses a whole face;
//  - FP64 compensated conservation sums of the face fluxes of both sides.
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
// Conservation sums (FP64, compensated).  Block b sums a fixed slice of the faces of
// both sides; a second pass adds the block partials in a fixed order (deterministic).
// ------------------------------------------------------------------------------------

struct Kahan {
    double s = 0.0, c = 0.0;
    __device__ void add(double x)
    {
        const double t = s + x;
        c += (fabs(s) >= fabs(x)) ? (s - t) + x : (x - t) + s;
        s = t;
    }
};

template <typename T>
__global__ void k_cons_partial(const T *__restrict__ Fs, const T *__restrict__ Fm,
                               const int32_t *__restrict__ fid_s,
                               const int32_t *__restrict__ fid_m,
                               const BasisConsts *__restrict__ basis, int NP, int nfaces,
                               int nfs, int nfm, double *__restrict__ part)
{
    // part[blk][v][3][2] (sum and compensation)
    __shared__ double red[256][2];
    const int P = NP * NP;
    for (int v = 0; v < 5; ++v) {
        Kahan ks, km, ka;
        for (int f = blockIdx.x * blockDim.x + threadIdx.x; f < nfaces;
             f += gridDim.x * blockDim.x) {
            const int cs = fid_s[f], cm = fid_m[f];
            for (int p = 0; p < P; ++p) {
                const double w = basis->w[p % NP] * basis->w[p / NP];
                const double a = w * (double)Fs[((size_t)v * P + p) * nfs + cs];
                const double b = w * (double)Fm[((size_t)v * P + p) * nfm + cm];
                ks.add(a);
                km.add(b);
                ka.add(fabs(a));
                ka.add(fabs(b));
            }
        }
        Kahan *acc[3] = {&ks, &km, &ka};
        for (int c = 0; c < 3; ++c) {
            red[threadIdx.x][0] = acc[c]->s;
            red[threadIdx.x][1] = acc[c]->c;
            __syncthreads();
            if (threadIdx.x == 0) {
                Kahan t;
                for (int i = 0; i < (int)blockDim.x; ++i) {
                    t.add(red[i][0]);
                    t.add(red[i][1]);
                }
                part[((size_t)blockIdx.x * 5 + v) * 6 + c * 2 + 0] = t.s;
                part[((size_t)blockIdx.x * 5 + v) * 6 + c * 2 + 1] = t.c;
            }
            __syncthreads();
        }
    }
}

__global__ void k_cons_final(const double *__restrict__ part, int nblk, double *__restrict__ out)
{
    const int e = threadIdx.x;  // (v, c)
    if (e >= 15) return;
    const int v = e / 3, c = e % 3;
    Kahan t;
    for (int b = 0; b < nblk; ++b) {
        t.add(part[((size_t)b * 5 + v) * 6 + c * 2 + 0]);
        t.add(part[((size_t)b * 5 + v) * 6 + c * 2 + 1]);
    }
    out[v * 3 + c] = t.s + t.c;
}

hipError_t launch_conservation(const Iface &f, const void *Fs, const void *Fm, double *d_out,
                               hipStream_t st)
{
    const int nblk = f.n_cons_blocks;
    if (f.d.precision == MORTAR_FP64)
        hipLaunchKernelGGL(k_cons_partial<double>, dim3(nblk), dim3(256), 0, st,
                           (const double *)Fs, (const double *)Fm, f.d_fid_s, f.d_fid_m,
                           f.d_basis, f.NP, f.F, f.d.n_face_static, f.d.n_face_moving, f.d_cons);
    else
        hipLaunchKernelGGL(k_cons_partial<float>, dim3(nblk), dim3(256), 0, st,
                           (const float *)Fs, (const float *)Fm, f.d_fid_s, f.d_fid_m,
                           f.d_basis, f.NP, f.F, f.d.n_face_static, f.d.n_face_moving, f.d_cons);
    hipLaunchKernelGGL(k_cons_final, dim3(1), dim3(64), 0, st, f.d_cons, nblk, d_out);
    return hipGetLastError();
}

}  // namespace mortar
