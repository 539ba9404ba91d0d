// Per-stage topology kernels of the mortar operator:
//  - FP64 projection matrices of the current s for inspection (the flux kernel
//    assembles its own copy in its prologue with the same routine);
//  - the device-side mortar sort (Sec. 4.4, Appendix A): sorted index array A and its
//    inverse map m, rebuilt when the displacement crosses a whole face;
//  - FP64 compensated conservation sums of the face fluxes of both sides.
#include <algorithm>
#include <mutex>

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
    __shared__ double work[assemble_scratch<NP>()];
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
        MORTAR_ASM_CASE(10) MORTAR_ASM_CASE(11) MORTAR_ASM_CASE(12) MORTAR_ASM_CASE(13)
        MORTAR_ASM_CASE(14) MORTAR_ASM_CASE(15) MORTAR_ASM_CASE(16)
    default: return hipErrorInvalidValue;
    }
#undef MORTAR_ASM_CASE
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// Pairing of every mortar of a row with its moving face, for inspection: the index
// relation the index map is built from, evaluated on the device for the current n.
// ------------------------------------------------------------------------------------

__global__ void k_pairing(int n_par, int nmod, int32_t *__restrict__ pair)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < 2 * n_par) pair[t] = moving_partner(t % n_par, t / n_par, nmod, n_par);
}

hipError_t launch_pairing(const Iface &f, hipStream_t st)
{
    const int64_t np = f.d.n_par;
    const int nmod = (int)(((f.n % np) + np) % np);
    const int total = 2 * f.d.n_par;
    hipLaunchKernelGGL(k_pairing, dim3((total + 255) / 256), dim3(256), 0, st, f.d.n_par, nmod,
                       f.d_pair);
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
    const int jt = moving_partner(ia, k, a.nmod, a.n_par);   // moving face of the mortar
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
// Conservation sums (FP64).  Each block sums a fixed set of (face, point) elements of
// one variable on one side with Neumaier compensation per thread; threads, waves and
// blocks are then combined in fixed orders (xor trees within waves, waves and blocks in
// sequence), so the result is deterministic.
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

// Plain double sum over a wave by a fixed xor tree (addition is commutative, so both
// partners of every step form the same value and the result is deterministic).
__device__ __forceinline__ double cons_wave_add(double x)
{
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) x += __shfl_xor(x, m);
    return x;
}

// Partial sums: block (bx, g) with g = v * 2 + side sums w_p w_q F and w_p w_q |F| of
// variable v on one side over the faces f = bx*256 + t + j*gridDim.x*256 and all points
// of each (consecutive threads read consecutive face columns, eight points in flight per
// thread).  Each thread accumulates with compensation; the few levels that combine
// threads and blocks add plain doubles in fixed orders.  part[(g * gridDim.x + bx)][2].
template <typename T>
__global__ __launch_bounds__(256) void k_cons_partial(const T *__restrict__ Fs,
                                                      const T *__restrict__ Fm,
                                                      const int32_t *__restrict__ fid_s,
                                                      const int32_t *__restrict__ fid_m,
                                                      const BasisConsts *__restrict__ basis,
                                                      int NP, int nfaces, int nfs, int nfm,
                                                      double *__restrict__ part)
{
    constexpr int PG = 8;
    __shared__ double red[4][2];
    __shared__ double wpq[kMaxNP * kMaxNP + PG];   // w_p w_q of point p, 0 past the last
    const int P = NP * NP;
    for (int p = threadIdx.x; p < P + PG; p += blockDim.x)
        wpq[p] = p < P ? basis->w[p % NP] * basis->w[p / NP] : 0.0;
    __syncthreads();
    const int g = blockIdx.y, v = g >> 1, side = g & 1;
    const int nf = side ? nfm : nfs;
    const T *F = (side ? Fm : Fs) + (size_t)v * P * nf;
    const int32_t *fid = side ? fid_m : fid_s;
    Neumaier sum, mag;
    for (int f = blockIdx.x * blockDim.x + threadIdx.x; f < nfaces; f += gridDim.x * blockDim.x) {
        const T *col = F + fid[f];
        for (int p0 = 0; p0 < P; p0 += PG) {
            T x[PG];
            // unconditional loads (a point past P rereads the last one, with weight 0), so
            // all of them are in flight at once
#pragma unroll
            for (int u = 0; u < PG; ++u) x[u] = col[(size_t)min(p0 + u, P - 1) * nf];
#pragma unroll
            for (int u = 0; u < PG; ++u) {
                const double y = wpq[p0 + u] * (double)x[u];
                sum.add(y);
                mag.add(fabs(y));
            }
        }
    }
    const double s1 = cons_wave_add(sum.s + sum.c), s2 = cons_wave_add(mag.s + mag.c);
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[wave][0] = s1;
        red[wave][1] = s2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, m = 0.0;
        for (int w2 = 0; w2 < (int)(blockDim.x >> 6); ++w2) {
            a += red[w2][0];
            m += red[w2][1];
        }
        double *o = part + ((size_t)g * gridDim.x + blockIdx.x) * 2;
        o[0] = a;
        o[1] = m;
    }
}

// Final pass: wave g = v * 2 + side adds its group's partials in a fixed order (each
// lane takes partials lane, lane + 64, ... with compensation, eight loads in flight
// before any is added, then the xor tree); out[v][0] = static integral, out[v][1] =
// moving integral, out[v][2] = sum of |terms|.
__device__ __forceinline__ void cons_final_block(const double *__restrict__ part, int nb,
                                                 double *__restrict__ out)
{
    __shared__ double res[10][2];
    const int g = threadIdx.x >> 6, lane = threadIdx.x & 63;
    constexpr int kAhead = 8;
    Neumaier a, m;
    for (int b0 = lane; b0 < nb; b0 += 64 * kAhead) {
        double va[kAhead], vm[kAhead];
#pragma unroll
        for (int k = 0; k < kAhead; ++k) {
            const int b = b0 + 64 * k;
            const size_t at = ((size_t)g * nb + (b < nb ? b : 0)) * 2;
            va[k] = part[at + 0];
            vm[k] = part[at + 1];
        }
#pragma unroll
        for (int k = 0; k < kAhead; ++k)
            if (b0 + 64 * k < nb) {
                a.add(va[k]);
                m.add(vm[k]);
            }
    }
    const double sa = cons_wave_add(a.s + a.c), sm = cons_wave_add(m.s + m.c);
    if (lane == 0) {
        res[g][0] = sa;
        res[g][1] = sm;
    }
    __syncthreads();
    if (threadIdx.x < 5) {
        const int vv = threadIdx.x;
        out[vv * 3 + 0] = res[vv * 2 + 0][0];
        out[vv * 3 + 1] = res[vv * 2 + 1][0];
        out[vv * 3 + 2] = res[vv * 2 + 0][1] + res[vv * 2 + 1][1];
    }
}

__global__ __launch_bounds__(640) void k_cons_final(const double *__restrict__ part, int nb,
                                                    double *__restrict__ out)
{
    cons_final_block(part, nb, out);
}

// The final pass of several interfaces in one launch, one workgroup each (the same
// arithmetic, so the same bits, as one k_cons_final per interface).
struct ConsFinalBatch {
    const double *part[kMaxConsBatch];
    double *out[kMaxConsBatch];
    int nb[kMaxConsBatch];
};

__global__ __launch_bounds__(640) void k_cons_final_batch(ConsFinalBatch b)
{
    cons_final_block(b.part[blockIdx.x], b.nb[blockIdx.x], b.out[blockIdx.x]);
}

// Conservation grid: blocks along the faces (one face per thread, every point of it;
// at most 1024 blocks, larger interfaces loop) for each of the 10 (variable, side) groups.
static int cons_face_blocks(int nfaces) { return std::max(1, std::min(1024, (nfaces + 255) / 256)); }

// Partials per (variable, side) group.
int cons_blocks(int P, int nfaces)
{
    (void)P;
    return cons_face_blocks(nfaces);
}

// Sums of several interfaces from the partials their fused flux launches wrote, one launch.
hipError_t launch_conservation_final_batch(const Iface *const *fs, double *const *outs, int n,
                                           hipStream_t st)
{
    if (n < 1 || n > kMaxConsBatch) return hipErrorInvalidValue;
    ConsFinalBatch b{};
    for (int i = 0; i < n; ++i) {
        b.part[i] = fs[i]->d_cons_wg;
        b.nb[i] = fs[i]->cons_nb;
        b.out[i] = outs[i];
    }
    hipLaunchKernelGGL(k_cons_final_batch, dim3(n), dim3(640), 0, st, b);
    return hipGetLastError();
}

// Whether a kernel (its host handle, as a graph's kernel node records it) is one of the
// conservation kernels, so that a captured stage can tell its flux nodes from them.
bool is_conservation_kernel(const void *func)
{
    return func == reinterpret_cast<const void *>(&k_cons_final) ||
           func == reinterpret_cast<const void *>(&k_cons_final_batch) ||
           func == reinterpret_cast<const void *>(&k_cons_partial<float>) ||
           func == reinterpret_cast<const void *>(&k_cons_partial<double>);
}

// Sums from the partials a fused flux launch wrote (one per workgroup and group).
hipError_t launch_conservation_final(const Iface &f, double *d_out, hipStream_t st)
{
    hipLaunchKernelGGL(k_cons_final, dim3(1), dim3(640), 0, st, f.d_cons_wg, f.cons_nb, d_out);
    return hipGetLastError();
}

// The pass over the flux arrays and the final reduction, with the partials in part
// (10 groups x cons_blocks() x 2 doubles).
static hipError_t launch_conservation_into(const Iface &f, const void *Fs, const void *Fm,
                                           double *part, double *d_out, hipStream_t st)
{
    const dim3 grid(cons_face_blocks(f.F), 10);
    const int nb = (int)grid.x;
    if (f.d.precision == MORTAR_FP64)
        hipLaunchKernelGGL(k_cons_partial<double>, grid, dim3(256), 0, st,
                           (const double *)Fs, (const double *)Fm, f.d_fid_s, f.d_fid_m,
                           f.d_basis, f.NP, f.F, f.d.n_face_static, f.d.n_face_moving, part);
    else
        hipLaunchKernelGGL(k_cons_partial<float>, grid, dim3(256), 0, st,
                           (const float *)Fs, (const float *)Fm, f.d_fid_s, f.d_fid_m,
                           f.d_basis, f.NP, f.F, f.d.n_face_static, f.d.n_face_moving, part);
    hipLaunchKernelGGL(k_cons_final, dim3(1), dim3(640), 0, st, part, nb, d_out);
    return hipGetLastError();
}

hipError_t launch_conservation(const Iface &f, const void *Fs, const void *Fm, double *d_out,
                               hipStream_t st)
{
    return launch_conservation_into(f, Fs, Fm, f.d_cons, d_out, st);
}

// ------------------------------------------------------------------------------------
// Conservation sums without any allocation: the partials of every interface of a call
// live in one file-scope device array (its own copy on every device the library runs
// on, held until the process ends).  Host code never passes the array's name to a
// kernel (in host code that name is not a device address): each device's address is
// looked up once, with that device current, and kept in the handle.
// ------------------------------------------------------------------------------------

static __device__ __align__(256) double scratch[kStaticConsIfaces * kStaticConsSlot];

static std::mutex g_scratch_mu;
static double *g_scratch_ptr[kMaxDevices] = {};

hipError_t static_cons_scratch(int device, double **out)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = static_cast<double *>(ptr);
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

hipError_t launch_conservation_static(const Iface &f, int slot, double *scratch_ptr,
                                      const void *Fs, const void *Fm, double *d_out, hipStream_t st)
{
    if (slot < 0 || slot >= kStaticConsIfaces || 20 * cons_face_blocks(f.F) > kStaticConsSlot)
        return hipErrorInvalidValue;
    return launch_conservation_into(f, Fs, Fm, scratch_ptr + (size_t)slot * kStaticConsSlot, d_out, st);
}

}  // namespace mortar
