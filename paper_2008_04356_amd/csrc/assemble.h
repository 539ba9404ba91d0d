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

// All Lagrange basis values l_j(xi) of the nodes (barycentric second form, exact at nodes).
template <int NP>
__device__ __forceinline__ void lagrange_row(const BasisConsts *__restrict__ c, double xi,
                                             double (&l)[NP])
{
    int hit = -1;
#pragma unroll
    for (int m = 0; m < NP; ++m)
        if (xi == c->x[m]) hit = m;
    if (hit >= 0) {
#pragma unroll
        for (int j = 0; j < NP; ++j) l[j] = (j == hit) ? 1.0 : 0.0;
        return;
    }
    double den = 0.0;
#pragma unroll
    for (int j = 0; j < NP; ++j) {
        l[j] = c->bw[j] / (xi - c->x[j]);
        den += l[j];
    }
    const double inv = 1.0 / den;
#pragma unroll
    for (int j = 0; j < NP; ++j) l[j] *= inv;
}

// Cooperative assembly by the threads of one block.  work: LDS scratch of at least
// 8*NP*NP doubles.  Writes Pf64/Pb64 (each [4][NP][NP], may be null) and PfT/PbT in the
// working precision (may be null).  Contains __syncthreads(): all threads must call it.
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
        // S_k[i][q] = sum_r tw_r Q_k[r][i] l_q(t_r);  Pb_k[j][q] = J_k sum_i Minv[j][i] S_k[i][q]
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
