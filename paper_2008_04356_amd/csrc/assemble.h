// FP64 assembly of the face->mortar and mortar->face projection matrices for a sub-face
// fraction s (Sec. 3.2: Eqs. for M, S and the two projections; Sec. 4.4: between face
// crossings only these operators change).  One device routine, used both by the fused
// flux kernel's prologue (every workgroup assembles its own copy while its first loads
// are in flight) and by the inspection kernel behind mortar_get_projection.
//
// Matrix order k: 0 static i_sub 0, 1 static i_sub 1, 2 moving i_sub 0 (upper part of
// the moving face), 3 moving i_sub 1 (lower part).  Pf_k[q][j] = l_j(xi_k(x_q)) (equal
// degree: the L2 projection is exact, so it is the interpolation matrix);
// Pb_k[j][q] = J_k sum_i Minv[j][i] S_k[i][q] with S_k[i][q] = int l_i(xi_k(z)) l_q(z) dz.
#pragma once

#include "mortar_internal.h"

namespace mortar {

// Face coordinate of mortar coordinate z on sub-interval k: xi = slope z + offset.
//   static i_sub 0: s z + (s - 1)        static i_sub 1: (1 - s) z + s
//   moving i_sub 0: s z + (1 - s)        moving i_sub 1: (1 - s) z - s
// The slope is the length ratio J_k of the sub-interval.
__device__ __forceinline__ void sub_map(int k, double s, double &slope, double &offset)
{
    switch (k) {
    case 0: slope = s; offset = s - 1.0; break;
    case 1: slope = 1.0 - s; offset = s; break;
    case 2: slope = s; offset = 1.0 - s; break;
    default: slope = 1.0 - s; offset = -s; break;
    }
}

// All Lagrange basis values l_j(xi) of the nodes, in the product form
// l_j(xi) = bw_j prod_{m != j} (xi - x_m) with the barycentric weights bw_j: prefix and
// suffix products, no division, exact (a zero factor) at the nodes themselves.
template <int NP>
__device__ __forceinline__ void lagrange_row(const BasisConsts *__restrict__ c, double xi,
                                             double (&l)[NP])
{
    double d[NP], pre[NP];
#pragma unroll
    for (int m = 0; m < NP; ++m) d[m] = xi - c->x[m];
    pre[0] = 1.0;
#pragma unroll
    for (int m = 1; m < NP; ++m) pre[m] = pre[m - 1] * d[m - 1];
    double suf = 1.0;
#pragma unroll
    for (int j = NP - 1; j >= 0; --j) {
        l[j] = c->bw[j] * (pre[j] * suf);
        suf *= d[j];
    }
}

// LDS scratch of the assembly, in doubles.
template <int NP> constexpr int assemble_scratch() { return 8 * NP * NP; }

// Cooperative assembly by the threads of one block: the basis rows at the mortar nodes
// (Pf) and at the Gauss points of each sub-interval (Q), then every entry of
// Pb_k = J_k Minv S_k with S_k[i][q] = sum_r tw_r Q_k[r][i] l_q(t_r) formed in place.
// work: LDS scratch of assemble_scratch<NP>() doubles.  Writes Pf64/Pb64 (each
// [4][NP][NP], may be null) and PfT/PbT in the working precision (may be null).
// Contains __syncthreads(): all threads must call it.
template <int NP, typename T>
__device__ void assemble_matrices(const BasisConsts *__restrict__ c, double s, double *work,
                                  double *Pf64, double *Pb64, T *PfT, T *PbT)
{
    constexpr int NN = NP * NP;
    double *Pf = work;            // [4][NP][NP]
    double *Q = work + 4 * NN;    // [4][NP(r)][NP(i)] = l_i(xi_k(t_r)) at the Gauss points
    const int tid = threadIdx.x;
    for (int e = tid; e < 8 * NP; e += blockDim.x) {
        const bool gauss_pts = e >= 4 * NP;
        const int row = gauss_pts ? e - 4 * NP : e;
        const int k = row / NP, q = row % NP;
        double a, b, l[NP];
        sub_map(k, s, a, b);
        lagrange_row<NP>(c, a * (gauss_pts ? c->t[q] : c->x[q]) + b, l);
        double *dst = (gauss_pts ? Q : Pf) + k * NN + q * NP;
#pragma unroll
        for (int j = 0; j < NP; ++j) dst[j] = l[j];
    }
    __syncthreads();
    for (int e = tid; e < 4 * NN; e += blockDim.x) {
        const int k = e / NN, j = (e % NN) / NP, q = e % NP;
        double a, b;
        sub_map(k, s, a, b);
        double acc = 0.0;
#pragma unroll
        for (int i = 0; i < NP; ++i) {
            double sk = 0.0;
#pragma unroll
            for (int r = 0; r < NP; ++r) sk += c->tw[r] * Q[k * NN + r * NP + i] * c->Lt[r * kMaxNP + q];
            acc += c->Minv[j * kMaxNP + i] * sk;
        }
        const double pb = a * acc;
        const double pf = Pf[e];
        if (Pb64) Pb64[e] = pb;
        if (Pf64) Pf64[e] = pf;
        if (PbT) PbT[e] = (T)pb;
        if (PfT) PfT[e] = (T)pf;
    }
    __syncthreads();
}

}  // namespace mortar
