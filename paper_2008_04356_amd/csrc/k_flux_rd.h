// Register-direct mortar-flux kernel: one wave per tile, both projections on the matrix
// cores, the pointwise fluxes computed straight from the matrix-core results.
//
// Operator: Sec. 3.3 steps 3-5 with the operators of Sec. 3.2, the same tile chain as the
// other flux kernels (k_flux.h).  A tile is 16 face slots of one line:
//   static slot f = face i0-1+f (slot 0 is the halo face),
//   moving slot f = face i0+f-n-1.
// Column f of the forward GEMM holds the two mortars (i0-1+f, 0) (rows 0..NP-1, node q)
// and (i0-1+f, 1) (rows NP..2NP-1).  On the static side these are the two sub-intervals
// of static slot f (matrices Pf0, Pf1).  On the moving side mortar (i0-1+f, 0) is the
// upper part of moving slot f-1 (Pf2) and (i0-1+f, 1) the lower part of moving slot f
// (Pf3), so the moving GEMM takes K = 2 NP: the first NP from the face data of slot f-1,
// brought over by a one-lane DPP shift inside each row of 16 lanes, the second NP from
// slot f itself.  With the matrix-core result layout every lane then holds both sides'
// values of the same mortar nodes for every variable and evaluates their Riemann + BR1
// fluxes in registers.  The back projection is a GEMM with K = the 2 NP mortar nodes of
// a column, whose B operand is exactly those flux registers (one more DPP shift for the
// moving side, whose upper mortar sits in the next column).  After the prologue only the
// conservation partials of the 4-byte launches go through LDS; in the lockstep launches
// (rd_lockstep) the waves of a workgroup meet at one barrier per round of tiles, so that
// they fetch the cache lines their neighbouring tiles share together.
//
// Precision (PREC): 0 runs the GEMMs in the element type (v_mfma_{f32,f64}_16x16x4).
// 1 / 2 round the GEMM operands to bf16 / fp16 (v_mfma_f32_16x16x16_{bf16,f16}, FP32
// accumulation; FP32 data; fp16 operands carry a power-of-two scale per wave, see
// rd_fp16_scale).  The rounded matrices no longer integrate exactly, so the
// back projection is then corrected per face line: with T the integral of the line's
// mortar fluxes (sum of J_k w_q F, FP64 accumulation of FP32 fluxes) and A the integral
// of the projected face flux (sum of w_j F_j), (T - A) / sum(w) is added to every node
// of the line.  This restores the line-by-line equality of the static and moving
// integrals (discrete conservation, Sec. 3.2) up to FP32 storage rounding.
#pragma once

#include <type_traits>

#include "assemble.h"
#include "flux_physics.h"
#include "k_flux.h"
#include "mortar_internal.h"

namespace mortar {

// Arrays of the register-direct kernel are addressed with 32-bit byte offsets through
// buffer descriptors: each stays at most kRdMaxBytes (the host checks), so the offset
// kRdOff of a masked-off lane is beyond every descriptor.  (The VALU kernels' kBufOff,
// 2 GiB, is inside a flux array of more than 2 GiB, which this kernel accepts.)
constexpr uint32_t kRdOff = (uint32_t)kRdMaxBytes;

typedef float rd_v4f __attribute__((ext_vector_type(4)));
typedef double rd_v4d __attribute__((ext_vector_type(4)));
typedef __bf16 rd_v4bf __attribute__((ext_vector_type(4)));
typedef _Float16 rd_v4h __attribute__((ext_vector_type(4)));

// Matrix-core operation of a precision mode.  Operand layouts: 16x16x4 (E = 1) lane l
// supplies A[l % 16][l / 16] and B[l / 16][l % 16]; 16x16x16 (E = 4) lane l supplies
// A[l % 16][4 (l / 16) + e] and B[4 (l / 16) + e][l % 16], e = 0..3.  Result: lane l,
// register r holds D[row(l / 16, r)][l % 16].
// Mortar nodes of the forward products: the A row R holds the coefficients of node
// node_of_row(R), chosen so that lane l, register r of a 16-row block gets node
// l / 16 + 4 r (rd_node) in every mode.  Register r of all lanes then holds nodes
// 4r .. 4r+3, and a register whose nodes all lie past the 2 NP of a column (every degree
// but N = 6 and 7) skips the pointwise flux as a whole; the same holds for the NP face
// nodes of the back projection's result (its stores and conservation terms).
template <typename T, int PREC> struct RdOp;
template <> struct RdOp<float, 0> {
    static constexpr int E = 1, KW = 4;
    using op_t = float;
    using acc_t = rd_v4f;
    __device__ static __forceinline__ op_t pack(const float *v) { return v[0]; }
    __device__ static __forceinline__ acc_t mma(op_t a, op_t b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    __device__ static __forceinline__ int row(int kq, int r) { return 4 * kq + r; }
    __device__ static __forceinline__ int node_of_row(int R) { return (R >> 2) + 4 * (R & 3); }
};
template <> struct RdOp<double, 0> {
    static constexpr int E = 1, KW = 4;
    using op_t = double;
    using acc_t = rd_v4d;
    __device__ static __forceinline__ op_t pack(const double *v) { return v[0]; }
    __device__ static __forceinline__ acc_t mma(op_t a, op_t b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    __device__ static __forceinline__ int row(int kq, int r) { return kq + 4 * r; }
    __device__ static __forceinline__ int node_of_row(int R) { return R; }
};
template <> struct RdOp<float, 1> {
    static constexpr int E = 4, KW = 16;
    using op_t = rd_v4bf;
    using acc_t = rd_v4f;
    __device__ static __forceinline__ op_t pack(const float *v)
    {
        op_t r;
#pragma unroll
        for (int e = 0; e < 4; ++e) r[e] = (__bf16)v[e];
        return r;
    }
    __device__ static __forceinline__ acc_t mma(op_t a, op_t b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
    }
    __device__ static __forceinline__ int row(int kq, int r) { return 4 * kq + r; }
    __device__ static __forceinline__ int node_of_row(int R) { return (R >> 2) + 4 * (R & 3); }
};
template <> struct RdOp<float, 2> {
    static constexpr int E = 4, KW = 16;
    using op_t = rd_v4h;
    using acc_t = rd_v4f;
    __device__ static __forceinline__ op_t pack(const float *v)
    {
        op_t r;
#pragma unroll
        for (int e = 0; e < 4; ++e) r[e] = (_Float16)v[e];
        return r;
    }
    __device__ static __forceinline__ acc_t mma(op_t a, op_t b, acc_t c)
    {
        return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
    }
    __device__ static __forceinline__ int row(int kq, int r) { return 4 * kq + r; }
    __device__ static __forceinline__ int node_of_row(int R) { return (R >> 2) + 4 * (R & 3); }
};

// Mortar node of lane group kq, register r (within a 16-row block); see RdOp.
__device__ __forceinline__ int rd_node(int kq, int r) { return kq + 4 * r; }
// Register r of block rb holds no mortar node of a column (2 NP nodes) in any lane.
template <int NP> __host__ __device__ constexpr bool rd_idle(int rb, int r) { return 16 * rb + 4 * r >= 2 * NP; }

template <int NP, bool NSV, bool MET, int KW, int WV>
struct RdCfg {
    static constexpr int V = NSV ? 20 : 5;                 // projected per side
    static constexpr int VS = V + (MET ? 4 : 0);           // static side adds the metrics
    static constexpr int NN = NP * NP;
    static constexpr int RB = (2 * NP + 15) / 16;          // 16-row blocks of mortar nodes
    static constexpr int KSF = (NP + KW - 1) / KW;         // static forward K steps
    static constexpr int KSM = (2 * NP + KW - 1) / KW;     // moving forward K steps
    static constexpr int KSB = RB * 16 / KW;               // backward K steps
    static constexpr int WAVES = WV;                       // waves per workgroup
    static constexpr int NT = 64 * WAVES;
};


// Value of lane - 1 (rd_left) or lane + 1 (rd_right) within each row of 16 lanes; the
// lane at the row's edge receives 0.
__device__ __forceinline__ int rd_shift_left(int x)
{
    return __builtin_amdgcn_update_dpp(0, x, 0x111, 0xF, 0xF, true);   // row_shr:1
}
__device__ __forceinline__ int rd_shift_right(int x)
{
    return __builtin_amdgcn_update_dpp(0, x, 0x101, 0xF, 0xF, true);   // row_shl:1
}
__device__ __forceinline__ float rd_left(float x) { return __int_as_float(rd_shift_left(__float_as_int(x))); }
__device__ __forceinline__ float rd_right(float x) { return __int_as_float(rd_shift_right(__float_as_int(x))); }
__device__ __forceinline__ double rd_left(double x)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    const unsigned lo = (unsigned)rd_shift_left((int)(unsigned)b);
    const unsigned hi = (unsigned)rd_shift_left((int)(unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ double rd_right(double x)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    const unsigned lo = (unsigned)rd_shift_right((int)(unsigned)b);
    const unsigned hi = (unsigned)rd_shift_right((int)(unsigned)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Cross-row exchanges without LDS (gfx950 permlane swaps): for each row of 16 lanes,
// rd_rows16 returns the pair (value of rows 2k, value of rows 2k+1) and rd_rows32 the pair
// (value of lanes l mod 32, value of lanes 32 + l mod 32), the same in both lanes of a
// pair; their sum equals x + shfl_xor(x, 16) (resp. 32) bit for bit (one commutative add).
__device__ __forceinline__ void rd_rows16(uint32_t x, uint32_t &a, uint32_t &b)
{
    const auto r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
    a = r[0];
    b = r[1];
}
__device__ __forceinline__ void rd_rows32(uint32_t x, uint32_t &a, uint32_t &b)
{
    const auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
    a = r[0];
    b = r[1];
}
// Sum of x over the four lanes col + 16 m (m = 0..3) of every column, in every lane.
__device__ __forceinline__ double rd_column_sum(double x)
{
#pragma unroll
    for (int step = 0; step < 2; ++step) {
        const unsigned long long u = (unsigned long long)__double_as_longlong(x);
        uint32_t alo, blo, ahi, bhi;
        if (step == 0) {
            rd_rows16((uint32_t)u, alo, blo);
            rd_rows16((uint32_t)(u >> 32), ahi, bhi);
        } else {
            rd_rows32((uint32_t)u, alo, blo);
            rd_rows32((uint32_t)(u >> 32), ahi, bhi);
        }
        const double p = __longlong_as_double((long long)(((unsigned long long)ahi << 32) | alo));
        const double q = __longlong_as_double((long long)(((unsigned long long)bhi << 32) | blo));
        x = p + q;
    }
    return x;
}
// Largest value of m over the wave, in every lane (non-negative m).
__device__ __forceinline__ float rd_wave_max(float m)
{
    uint32_t a, b;
    rd_rows16(__float_as_uint(m), a, b);
    m = fmaxf(__uint_as_float(a), __uint_as_float(b));
    rd_rows32(__float_as_uint(m), a, b);
    m = fmaxf(__uint_as_float(a), __uint_as_float(b));
    // within each row of 16 lanes: rotations by 8, 4, 2, 1
    m = fmaxf(m, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(m), 0x128, 0xF, 0xF, false)));
    m = fmaxf(m, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(m), 0x124, 0xF, 0xF, false)));
    m = fmaxf(m, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(m), 0x122, 0xF, 0xF, false)));
    m = fmaxf(m, __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(m), 0x121, 0xF, 0xF, false)));
    return m;
}

// fp16 operands: a power-of-two scale per wave and operand set keeps the values in the
// normal range of fp16 (surface elements of fine meshes push fluxes below 6e-5, where
// fp16 loses precision and then flushes to zero).  Scaling by powers of two is exact, so
// the result is unscaled exactly afterwards.  Returns the scale for values of magnitude
// up to m (the largest magnitude in this lane); maps the wave's largest into [1, 2).
__device__ __forceinline__ float rd_fp16_scale(float m, float &inv)
{
    m = rd_wave_max(m);
    const int ex = (int)((__float_as_uint(m) >> 23) & 0xFF) - 127;
    if (!(m > 0.0f) || ex > 126 || ex < -126) {   // zero, non-finite or extreme: no scaling
        inv = 1.0f;
        return 1.0f;
    }
    inv = __uint_as_float((uint32_t)(127 + ex) << 23);
    return __uint_as_float((uint32_t)(127 - ex) << 23);
}

// Workgroups of this workgroup's XCD (blockIdx.x % kXcds), and this workgroup's place
// among them after a rotation by rot (0 <= rot < that count).  A batch rotates the order
// from one interface to the next (rd_next_rot), so that the workgroups that take the
// last, partial round of one interface come last in the next one's.
__device__ __forceinline__ int rd_xcd_workgroups()
{
    const int g = gridDim.x, xcd = blockIdx.x % kXcds;
    return g / kXcds + ((g % kXcds) > xcd ? 1 : 0);
}
__device__ __forceinline__ int rd_place(int nwg, int rot) { return (blockIdx.x / kXcds + rot) % nwg; }

// The rotation for the next interface, given that of this one: a share of len tiles
// taken unit units per workgroup and round leaves its last round to the e workgroups at
// places 0 .. e-1; the next interface starts its places at the workgroup after them.
__device__ __forceinline__ int rd_next_rot(int len, int unit, int rot)
{
    const int nwg = rd_xcd_workgroups();
    const int e = ((max(len, 0) % (nwg * unit)) + unit - 1) / unit;   // 0 <= e <= nwg
    return (rot - e + nwg) % nwg;
}

// Persistent schedule at wave granularity, with the XCD split of TileCursor: XCD x owns
// the contiguous eighth of the tiles, and the waves of the workgroups on that XCD take
// them in turn.  Requires gridDim.x >= min(8, n) so that every XCD's share has workers.
struct WaveCursor {
    int k, limit, stride;
    __device__ WaveCursor(int n, int waves, int wave, int rot = 0)
    {
        const int xcd = blockIdx.x % kXcds;
        const int nwg = rd_xcd_workgroups();
        stride = nwg * waves;
        const int per = (n + kXcds - 1) / kXcds;
        const int base = xcd * per;
        limit = min(n, base + per);
        k = base + rd_place(nwg, rot) * waves + wave;
    }
    // the rotation for the next interface of a batch
    static __device__ int next_rot(int n, int waves, int rot)
    {
        const int per = (n + kXcds - 1) / kXcds;
        const int base = (blockIdx.x % kXcds) * per;
        return rd_next_rot(min(n, base + per) - base, waves, rot);
    }
    __device__ bool valid() const { return k < limit; }
    // some wave of this workgroup has a tile in the current round (the same answer for
    // every wave of the workgroup)
    __device__ bool round_valid(int wave) const { return k - wave < limit; }
    __device__ int tile() const { return k; }
    __device__ void next() { k += stride; }
};

// The wave cursor of the out-of-phase lockstep groups: each XCD's eighth of the tiles is
// cut in two halves, the first group (waves 0 .. waves/2 - 1) takes the first half and the
// second group the second, so that the two groups, which run half a round apart, share
// no cache lines except where the halves meet.  A round is run while the first group's
// first wave has a tile (the first half is never the shorter), the same answer for every
// wave of the workgroup.
struct HalfCursor {
    int k, limit, stride, first, first_limit;
    __device__ HalfCursor(int n, int waves, int wave, int rot = 0)
    {
        const int xcd = blockIdx.x % kXcds;
        const int nwg = rd_xcd_workgroups();
        const int per = (n + kXcds - 1) / kXcds;
        const int base = min(n, xcd * per);
        const int lim = min(n, base + per);
        const int mid = base + (lim - base + 1) / 2;
        const int hw = waves / 2;
        const int grp = wave < hw ? 0 : 1;
        const int place = rd_place(nwg, rot);
        stride = nwg * hw;
        first = base + place * hw;
        first_limit = mid;
        k = (grp ? mid : base) + place * hw + (wave - grp * hw);
        limit = grp ? lim : mid;
    }
    // the rotation for the next interface of a batch: the rounds follow the first half
    static __device__ int next_rot(int n, int waves, int rot)
    {
        const int per = (n + kXcds - 1) / kXcds;
        const int base = min(n, (blockIdx.x % kXcds) * per);
        const int lim = min(n, base + per);
        return rd_next_rot((lim - base + 1) / 2, waves / 2, rot);
    }
    __device__ bool valid() const { return k < limit; }
    __device__ bool round_valid(int) const { return first < first_limit; }
    __device__ int tile() const { return k; }
    __device__ void next()
    {
        k += stride;
        first += stride;
    }
};

// One interface: every workgroup assembles the stage's matrices, then its waves take
// tiles from the interface's wave cursor.  work: LDS of 8 NP^2 doubles; mats: 8 NP^2
// element-type values; wq: NP doubles.  Contains __syncthreads (all threads call it).
// Launches with 4-byte data (FP32, bf16, fp16) also write the conservation partials of
// the values they store: every lane adds w_p w_q F and its magnitude per (variable, side) into
// its own LDS slots (acc, [20][NT] doubles), and at the end of the interface the
// workgroup adds its lanes' slots in a fixed order (red: 320 doubles of scratch) into
// a.cons (layout of FluxArgs).
// LIFT: the BR1 lifting surface term instead of the flux (Euler-shaped: states and
// metrics in, no gradients): at every mortar node the average of both sides' states times
// each component of the static unit normal and the surface element, 15 values
// (component d, variable v at plane 5 d + v) back-projected onto both sides.
template <typename T, int NP, bool NSV, bool MET, int RIEM, int PREC, int WV, bool LIFT = false>
__device__ __forceinline__ int rd_interface(const FluxArgs<T> &a, double *work, T *mats, double *wq,
                                            double *acc, double *red, int rot = 0)
{
    static_assert(!LIFT || (!NSV && PREC == 0), "lifting: states only, element-type products");
    constexpr int NOUT = LIFT ? 15 : 5;      // output planes per side
    using Op = RdOp<T, PREC>;
    using C = RdCfg<NP, NSV, MET, Op::KW, WV>;
    using op_t = typename Op::op_t;
    using acc_t = typename Op::acc_t;
    constexpr int V = C::V, VS = C::VS, NN = C::NN, RB = C::RB, E = Op::E, KW = Op::KW;
    constexpr int KSF = C::KSF, KSM = C::KSM, KSB = C::KSB, P = NN;
    constexpr int LF = KSF * E, LM = KSM * E;              // loaded values per lane and var
    static_assert(C::NT == 64 * WV, "launch bounds");
    static_assert(NP <= 16, "one 16-row block of face nodes in the back projection");

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int col = lane & 15;               // slot of this lane
    const int kq = lane >> 4;                // operand K group / result row group

    assemble_matrices<NP, T>(a.basis, a.s, work, nullptr, nullptr, mats, mats + 4 * NN);
    if (tid < NP) wq[tid] = a.basis->w[tid];
    __syncthreads();

    auto kidx = [&](int ks, int e) { return ks * KW + (E == 1 ? kq : 4 * kq + e); };

    // ---- A operands, kept in registers for the whole launch ----------------------------
    op_t Afs[RB][KSF], Afm[RB][KSM], Abs[KSB], Abm[KSB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) {
        const int row = 16 * rb + Op::node_of_row(col);   // node of this lane's A row
#pragma unroll
        for (int ks = 0; ks < KSF; ++ks) {
            T x[4] = {0, 0, 0, 0};
            float f[4] = {0, 0, 0, 0};
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int j = kidx(ks, e);
                if (j < NP && row < NP) x[e] = mats[0 * NN + row * NP + j];
                if (j < NP && row >= NP && row < 2 * NP) x[e] = mats[1 * NN + (row - NP) * NP + j];
                f[e] = (float)x[e];
            }
            if constexpr (PREC == 0) Afs[rb][ks] = Op::pack(x);
            else Afs[rb][ks] = Op::pack(f);
        }
#pragma unroll
        for (int ks = 0; ks < KSM; ++ks) {
            T x[4] = {0, 0, 0, 0};
            float f[4] = {0, 0, 0, 0};
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int k = kidx(ks, e);
                if (k < NP && row < NP) x[e] = mats[2 * NN + row * NP + k];
                if (k >= NP && k < 2 * NP && row >= NP && row < 2 * NP)
                    x[e] = mats[3 * NN + (row - NP) * NP + (k - NP)];
                f[e] = (float)x[e];
            }
            if constexpr (PREC == 0) Afm[rb][ks] = Op::pack(x);
            else Afm[rb][ks] = Op::pack(f);
        }
    }
    // back projection: A row R = col holds face node j = node_of_row(col) (so that lane
    // group kq, register r of the result holds face node rd_node(kq, r)); column rho =
    // the mortar node supplied in K step kb
    auto bsrc = [&](int kb, int e, int &rb, int &r) {
        rb = E == 1 ? kb / 4 : kb;
        r = E == 1 ? kb % 4 : e;
    };
#pragma unroll
    for (int kb = 0; kb < KSB; ++kb) {
        T xs[4] = {0, 0, 0, 0}, xm[4] = {0, 0, 0, 0};
        float fs[4] = {0, 0, 0, 0}, fm[4] = {0, 0, 0, 0};
#pragma unroll
        for (int e = 0; e < E; ++e) {
            int rb, r;
            bsrc(kb, e, rb, r);
            const int rho = 16 * rb + rd_node(kq, r);
            const int jn = Op::node_of_row(col);
            if (jn < NP && rho < 2 * NP) {
                const int k = rho < NP ? 0 : 1;
                const int q = rho - k * NP;
                xs[e] = mats[4 * NN + k * NN + jn * NP + q];
                xm[e] = mats[4 * NN + (2 + k) * NN + jn * NP + q];
            }
            fs[e] = (float)xs[e];
            fm[e] = (float)xm[e];
        }
        if constexpr (PREC == 0) {
            Abs[kb] = Op::pack(xs);
            Abm[kb] = Op::pack(xm);
        } else {
            Abs[kb] = Op::pack(fs);
            Abm[kb] = Op::pack(fm);
        }
    }
    // mortar-node rows of this lane and their quadrature weights J_k w_q (the same on
    // both sides: J = s for mortar (., 0) = moving upper part, 1 - s for (., 1))
    int rrow[RB][4];
    double cw[RB][4];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int rho = 16 * rb + rd_node(kq, r);
            rrow[rb][r] = rho;
            cw[rb][r] = rho < NP ? a.s * wq[rho] : (rho < 2 * NP ? (1.0 - a.s) * wq[rho - NP] : 0.0);
        }
    double wj[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int j = rd_node(kq, r);
        wj[r] = j < NP ? wq[j] : 0.0;
    }
    // conservation partials written with the fluxes in the 4-byte modes (the FP64
    // kernel's registers are already spent: its partials come from a pass)
    constexpr bool FUSE = sizeof(T) == 4 && !LIFT;
    if constexpr (FUSE) {
#pragma unroll
        for (int k = 0; k < 20; ++k) acc[k * C::NT + tid] = 0.0;
    }

    const int np_ = a.n_par;
    const int nmod = a.nmod;
    // buffer resources of the arrays (each at most kRdMaxBytes; the host checks this)
    const int pbytes_s = (int)((size_t)P * a.nfs * sizeof(T));
    const int pbytes_m = (int)((size_t)P * a.nfm * sizeof(T));
    const buf_rsrc_t rU_s = buf_rsrc(a.Us, 5u * (uint32_t)pbytes_s);
    const buf_rsrc_t rU_m = buf_rsrc(a.Um, 5u * (uint32_t)pbytes_m);
    const buf_rsrc_t rG_s = buf_rsrc(a.Gs, NSV ? 15u * (uint32_t)pbytes_s : 0u);
    const buf_rsrc_t rG_m = buf_rsrc(a.Gm, NSV ? 15u * (uint32_t)pbytes_m : 0u);
    const buf_rsrc_t rMet = buf_rsrc(a.met, MET ? 4u * (uint32_t)pbytes_s : 0u);
    const buf_rsrc_t rF_s = buf_rsrc(a.Fs, (uint32_t)NOUT * (uint32_t)pbytes_s);
    const buf_rsrc_t rF_m = buf_rsrc(a.Fm, (uint32_t)NOUT * (uint32_t)pbytes_m);

    // ---- per-tile operand fetch ---------------------------------------------------
    // One 32-bit byte offset per K value, shared by all variables (the variable's plane
    // is the scalar offset).  Padding K values and columns outside the tile read node 0
    // of a valid face: their A entries are zero or their columns are never used.
    T ls[VS][LF], lm[V][LM];
    // column of this lane's static / moving face in tile g: every lane loads (lanes past
    // the tile the column of the tile's last face), so the number of memory operations
    // between a lookup and its use does not depend on the path taken
    auto col_s = [&](const TileGeom &g) {
        int i = g.i0 - 1 + min(col, g.nf);
        if (i < 0) i += np_;
        return a.fid_s[(size_t)g.row * np_ + i];
    };
    auto col_m = [&](const TileGeom &g) {
        int jt = g.i0 + min(col, g.nf) - nmod - 1;
        if (jt < 0) jt += np_;
        return a.fid_m[(size_t)g.row * np_ + jt];
    };
    // The loads of a tile are issued in the order of their first use: both sides'
    // states and the metrics, then the static and the moving gradients.  Vector-memory
    // loads complete in issue order, so the projections of the states and the convective
    // flux wait only for the first of them.  (Issuing the moving gradients only after
    // the convective flux, which keeps fewer loads outstanding than the wave's counter
    // holds, left their latency exposed and was slower.)
    uint32_t os[LF], om[LM];
    auto offsets = [&](const TileGeom &g, int cs_, int cm_) {
        const uint32_t cs = (uint32_t)cs_, cm = (uint32_t)cm_, line = (uint32_t)(NP * g.pp);
#pragma unroll
        for (int ks = 0; ks < KSF; ++ks)
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int j = kidx(ks, e);
                os[ks * E + e] = ((line + (j < NP ? j : 0)) * (uint32_t)a.nfs + cs) * (uint32_t)sizeof(T);
            }
#pragma unroll
        for (int ks = 0; ks < KSM; ++ks)
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int k = kidx(ks, e);
                const int j = k < NP ? k : (k < 2 * NP ? k - NP : 0);
                om[ks * E + e] = ((line + j) * (uint32_t)a.nfm + cm) * (uint32_t)sizeof(T);
            }
    };
    auto fetch_s = [&](int v0, int v1) {
#pragma unroll
        for (int v = v0; v < v1; ++v) {
            const buf_rsrc_t &rs = v < 5 ? rU_s : (v < V ? rG_s : rMet);
            const int pv = v < 5 ? v : (v < V ? v - 5 : v - V);
#pragma unroll
            for (int q = 0; q < LF; ++q) ls[v][q] = buf_load<T>(rs, os[q], (int)((uint32_t)pv * (uint32_t)pbytes_s));
        }
    };
    auto fetch_m = [&](int v0, int v1) {
#pragma unroll
        for (int v = v0; v < v1; ++v) {
            const buf_rsrc_t &rs = v < 5 ? rU_m : rG_m;
            const int pv = v < 5 ? v : v - 5;
#pragma unroll
            for (int q = 0; q < LM; ++q) lm[v][q] = buf_load<T>(rs, om[q], (int)((uint32_t)pv * (uint32_t)pbytes_m));
        }
    };
    auto proj_s = [&](const T (&b)[LF], acc_t (&d)[RB]) {
        float sc = 1.0f, inv = 1.0f;
        if constexpr (PREC == 2) {
            float m = 0.0f;
#pragma unroll
            for (int q = 0; q < LF; ++q) m = fmaxf(m, fabsf((float)b[q]));
            sc = rd_fp16_scale(m, inv);
        }
        op_t bo[KSF];
#pragma unroll
        for (int ks = 0; ks < KSF; ++ks) {
            if constexpr (PREC == 0) bo[ks] = Op::pack(&b[ks * E]);
            else {
                float f[4];
#pragma unroll
                for (int e = 0; e < E; ++e) f[e] = (float)b[ks * E + e] * sc;
                bo[ks] = Op::pack(f);
            }
        }
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            acc_t acc = {0, 0, 0, 0};
#pragma unroll
            for (int ks = 0; ks < KSF; ++ks) acc = Op::mma(Afs[rb][ks], bo[ks], acc);
            if constexpr (PREC == 2) {
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[r] *= inv;
            }
            d[rb] = acc;
        }
    };
    auto proj_m = [&](const T (&b)[LM], acc_t (&d)[RB]) {
        float sc = 1.0f, inv = 1.0f;
        if constexpr (PREC == 2) {
            float m = 0.0f;     // the shifted values are other lanes' own values
#pragma unroll
            for (int q = 0; q < LM; ++q) m = fmaxf(m, fabsf((float)b[q]));
            sc = rd_fp16_scale(m, inv);
        }
        op_t bo[KSM];
#pragma unroll
        for (int ks = 0; ks < KSM; ++ks) {
            T x[4];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const T own = b[ks * E + e];
                const T sh = rd_left(own);
                x[e] = kidx(ks, e) < NP ? sh : own;
            }
            if constexpr (PREC == 0) bo[ks] = Op::pack(x);
            else {
                float f[4];
#pragma unroll
                for (int e = 0; e < E; ++e) f[e] = (float)x[e] * sc;
                bo[ks] = Op::pack(f);
            }
        }
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            acc_t acc = {0, 0, 0, 0};
#pragma unroll
            for (int ks = 0; ks < KSM; ++ks) acc = Op::mma(Afm[rb][ks], bo[ks], acc);
            if constexpr (PREC == 2) {
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[r] *= inv;
            }
            d[rb] = acc;
        }
    };

    // Register budget: the waves hide each other's latency (two per SIMD for Navier-Stokes,
    // more for Euler), so a tile keeps few values live.  The gradients of one side are
    // projected only when its viscous flux is evaluated, and the pointwise fluxes of the
    // lane's mortar nodes are evaluated one after the other: an empty asm statement that
    // takes the previous node's flux and redefines the next node's inputs stops the
    // compiler from interleaving all of them (which multiplies the live temporaries).
    // A tile's loads are issued at its start and the other waves of the SIMD cover their
    // latency.  The face columns of the next tile are looked up at the start of the
    // current one, before its loads: vector-memory operations complete in issue order,
    // so the current tile's loads (waited for anyway) retire the lookup, while a lookup
    // issued after the previous tile's stores would also wait for them.
    // Lockstep launches (rd_lockstep: 4-byte data, Navier-Stokes, and Euler with enough
    // nodes per line): the waves of the workgroup go through the rounds of tiles
    // together: every wave runs every round (a wave without a tile in a round computes
    // tile 0 and stores nothing), and one barrier per round and wave keeps them together,
    // in two groups out of phase (kRdPingPong) that take their tiles from the two halves
    // of the XCD's share (HalfCursor).  This fetches the lines neighbouring tiles share
    // once and writes back each line once.  The other launches run their waves freely
    // (FP64 has one or two waves per SIMD and no conservation slots; the smaller Euler
    // launches keep three or four waves per SIMD in four-wave workgroups).
    constexpr bool LOCKSTEP = LIFT ? WV == kRdLockWaves : rd_lockstep((int)sizeof(T), NSV, NP);
    using Cursor = std::conditional_t<LOCKSTEP && kRdPingPong && kRdSplitHalves, HalfCursor, WaveCursor>;
    Cursor cur(a.n_tiles, C::WAVES, wave, rot);
    bool more = LOCKSTEP ? cur.round_valid(wave) : cur.valid();
    bool mine = cur.valid();
    TileGeom g = tile_geom(a, mine ? cur.tile() : 0, NP);
    int cs_c = col_s(g), cm_c = col_m(g);
    // the first columns are waited for here, so that the loop is entered, like every later
    // iteration, with no lookup outstanding
    asm volatile("" ::"v"(cs_c), "v"(cm_c));
    while (more) {
        const TileGeom gc = g;
        const bool live_tile = mine;
        cur.next();
        more = LOCKSTEP ? cur.round_valid(wave) : cur.valid();
        mine = cur.valid();
        g = tile_geom(a, mine ? cur.tile() : 0, NP);   // tile 0: a dead lookup
        // every wave passes one barrier per round: here, or (first group of the
        // ping-pong) once the round's loads are issued
        if constexpr (LOCKSTEP) {
            if (!kRdPingPong || wave >= WV / 2) __builtin_amdgcn_s_barrier();
        }
        const int cs_n = col_s(g), cm_n = col_m(g);
        // this tile's columns: the static face of slot col and the moving face of slot
        // col are also the faces this lane writes
        const int oc_s = cs_c, oc_m = cm_c;
        offsets(gc, oc_s, oc_m);
        fetch_s(0, 5);
        fetch_s(V, VS);
        fetch_m(0, 5);
        fetch_s(5, V);
        fetch_m(5, V);
        // every load of the tile is issued before the first is used
        __builtin_amdgcn_sched_barrier(0);
        if constexpr (LOCKSTEP && kRdPingPong) {
            if (wave < WV / 2) __builtin_amdgcn_s_barrier();
        }
        cs_c = cs_n;
        cm_c = cm_n;
        acc_t QL[5][RB], QR[5][RB], MT[MET ? 4 : 1][RB];
#pragma unroll
        for (int v = 0; v < 5; ++v) {
            proj_s(ls[v], QL[v]);
            proj_m(lm[v], QR[v]);
        }
        if constexpr (MET) {
#pragma unroll
            for (int c = 0; c < 4; ++c) proj_s(ls[V + c], MT[c]);
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (rd_idle<NP>(rb, r)) continue;
                    T nx = MT[0][rb][r], ny = MT[1][rb][r], nz = MT[2][rb][r];
                    unit_normal(nx, ny, nz);
                    MT[0][rb][r] = nx;
                    MT[1][rb][r] = ny;
                    MT[2][rb][r] = nz;
                }
        }

        // rows of this lane that are mortar nodes the tile needs: mortar (i0-1+col, 0)
        // for col >= 1, mortar (i0-1+col, 1) for every live column
        const bool live = col <= gc.nf;
        bool use[RB][4];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int rho = rrow[rb][r];
                use[rb][r] = live && (rho < NP ? col >= 1 : rho < 2 * NP);
            }
        auto normal = [&](int rb, int r, T &nx, T &ny, T &nz) {
            nx = a.nx;
            ny = a.ny;
            nz = a.nz;
            if constexpr (MET) {
                nx = MT[0][rb][r];
                ny = MT[1][rb][r];
                nz = MT[2][rb][r];
            }
        };
        // ---- flux at the lane's mortar nodes --------------------------------------------
        // Rows that are not needed mortar nodes (padding rows, the halo column's first
        // mortar, columns past the tile) hold values that may be anything, even
        // non-finite; their fluxes are replaced by exact zeros below, and no other row or
        // column ever reads them.
        T FR[NOUT][RB][4];
        T Fprev[5] = {0, 0, 0, 0, 0};
        if constexpr (LIFT) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (rd_idle<NP>(rb, r)) {
#pragma unroll
                        for (int o = 0; o < NOUT; ++o) FR[o][rb][r] = T(0);
                        continue;
                    }
                    T n[3], dS = a.dS;
                    normal(rb, r, n[0], n[1], n[2]);
                    if constexpr (MET) dS = MT[3][rb][r];
                    // rows that are not needed mortar nodes may hold anything (the unit
                    // normal of a zero padding row is not finite): selected, not multiplied
#pragma unroll
                    for (int v = 0; v < 5; ++v) {
                        const T avg = T(0.5) * (T(QL[v][rb][r]) + T(QR[v][rb][r])) * dS;
#pragma unroll
                        for (int d = 0; d < 3; ++d) FR[5 * d + v][rb][r] = use[rb][r] ? avg * n[d] : T(0);
                    }
                }
        } else {
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if (rd_idle<NP>(rb, r)) {            // no mortar node in any lane
#pragma unroll
                    for (int v = 0; v < 5; ++v) FR[v][rb][r] = T(0);
                    continue;
                }
                T UL[5], UR[5], F[5], nx, ny, nz;
#pragma unroll
                for (int v = 0; v < 5; ++v) {
                    UL[v] = T(QL[v][rb][r]);
                    UR[v] = T(QR[v][rb][r]);
                }
                if (rb + r > 0)
                    asm volatile("" : "+v"(UL[0]), "+v"(UL[1]), "+v"(UL[2]), "+v"(UL[3]), "+v"(UL[4]),
                                      "+v"(UR[0]), "+v"(UR[1]), "+v"(UR[2]), "+v"(UR[3]), "+v"(UR[4])
                                    : "v"(Fprev[0]), "v"(Fprev[1]), "v"(Fprev[2]), "v"(Fprev[3]), "v"(Fprev[4]));
                normal(rb, r, nx, ny, nz);
                convective_flux<T, RIEM>(UL, UR, nx, ny, nz, a.gas, F);
#pragma unroll
                for (int v = 0; v < 5; ++v) FR[v][rb][r] = Fprev[v] = F[v];
            }
        // BR1: minus half the viscous flux of each side, one side's gradients at a time
        if constexpr (NSV) {
#pragma unroll
            for (int sd = 0; sd < 2; ++sd) {
                acc_t GQ[15][RB];
#pragma unroll
                for (int gg = 0; gg < 15; ++gg) {
                    if (sd == 0) proj_s(ls[5 + gg], GQ[gg]);
                    else proj_m(lm[5 + gg], GQ[gg]);
                }

#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        if (rd_idle<NP>(rb, r)) continue;
                        T U[5], G[15], Fv[5], nx, ny, nz;
#pragma unroll
                        for (int v = 0; v < 5; ++v) U[v] = T(sd == 0 ? QL[v][rb][r] : QR[v][rb][r]);
#pragma unroll
                        for (int gg = 0; gg < 15; ++gg) G[gg] = T(GQ[gg][rb][r]);
                        asm volatile("" : "+v"(G[0]), "+v"(G[1]), "+v"(G[2]), "+v"(G[3]), "+v"(G[4]),
                                          "+v"(G[5]), "+v"(G[6]), "+v"(G[7]), "+v"(G[8]), "+v"(G[9]),
                                          "+v"(G[10]), "+v"(G[11]), "+v"(G[12]), "+v"(G[13]),
                                          "+v"(G[14]), "+v"(U[0]), "+v"(U[4])
                                        : "v"(Fprev[1]), "v"(Fprev[2]), "v"(Fprev[3]), "v"(Fprev[4]));
                        normal(rb, r, nx, ny, nz);
                        viscous_flux(U, G, nx, ny, nz, a.gas, Fv);
#pragma unroll
                        for (int v = 1; v < 5; ++v) Fprev[v] = FR[v][rb][r] -= T(0.5) * Fv[v];
                    }
            }
        }
        // surface element; rows that are not needed mortar nodes contribute nothing
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if (rd_idle<NP>(rb, r)) continue;          // already zero
                T dS = a.dS;
                if constexpr (MET) dS = MT[3][rb][r];
#pragma unroll
                for (int v = 0; v < 5; ++v) FR[v][rb][r] = use[rb][r] ? FR[v][rb][r] * dS : T(0);
            }
        }   // flux (not LIFT)

        // ---- back projection onto both sides ----------------------------------------
        const bool out_s = live_tile && col >= 1 && col <= gc.nf;   // static face i0-1+col
        const bool out_m = live_tile && col < gc.nf;                // moving face of slot col
        const double wpp = FUSE ? wq[gc.pp] : 0.0;                 // weight of the line
        const uint32_t line = (uint32_t)(NP * gc.pp);
#pragma unroll
        for (int v = 0; v < NOUT; ++v) {
            // moving face of slot col: lower part = mortar (i0-1+col, 1) of this column,
            // upper part = mortar (i0+col, 0) of the next column
            T FM[RB][4];
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (rd_idle<NP>(rb, r)) {
                        FM[rb][r] = T(0);
                        continue;
                    }
                    const T nxt = rd_right(FR[v][rb][r]);
                    FM[rb][r] = rrow[rb][r] < NP ? nxt : FR[v][rb][r];
                }
            float sc = 1.0f, inv = 1.0f;
            if constexpr (PREC == 2) {
                float m = 0.0f;    // FM holds values of this wave's FR
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                    for (int r = 0; r < 4; ++r) m = fmaxf(m, fabsf((float)FR[v][rb][r]));
                sc = rd_fp16_scale(m, inv);
            }
            acc_t ds = {0, 0, 0, 0}, dm = {0, 0, 0, 0};
#pragma unroll
            for (int kb = 0; kb < KSB; ++kb) {
                if (E == 1 && rd_idle<NP>(kb / 4, kb % 4)) continue;   // a zero B operand
                T xs[4], xm[4];
                float fs[4], fm[4];
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    int rb, r;
                    bsrc(kb, e, rb, r);
                    xs[e] = FR[v][rb][r];
                    xm[e] = FM[rb][r];
                    fs[e] = (float)xs[e] * sc;
                    fm[e] = (float)xm[e] * sc;
                }
                if constexpr (PREC == 0) {
                    ds = Op::mma(Abs[kb], Op::pack(xs), ds);
                    dm = Op::mma(Abm[kb], Op::pack(xm), dm);
                } else {
                    ds = Op::mma(Abs[kb], Op::pack(fs), ds);
                    dm = Op::mma(Abm[kb], Op::pack(fm), dm);
                }
            }
            if constexpr (PREC == 2) {
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    ds[r] *= inv;
                    dm[r] *= inv;
                }
            }
            if constexpr (PREC != 0) {
                double Ts = 0.0, Tm = 0.0, As = 0.0, Am = 0.0;
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        Ts += cw[rb][r] * (double)FR[v][rb][r];
                        Tm += cw[rb][r] * (double)FM[rb][r];
                    }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (4 * r >= NP) continue;             // no face node in any lane
                    As += wj[r] * (double)ds[r];
                    Am += wj[r] * (double)dm[r];
                }
                // sum over the four row groups of the column (lanes col + 16 m)
                Ts = rd_column_sum(Ts);
                Tm = rd_column_sum(Tm);
                As = rd_column_sum(As);
                Am = rd_column_sum(Am);
                const float corr_s = (float)(0.5 * (Ts - As));   // the weights sum to 2
                const float corr_m = (float)(0.5 * (Tm - Am));
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    ds[r] += corr_s;
                    dm[r] += corr_m;
                }
            }
            if constexpr (FUSE) {
                // the stored values (rounded to the element type), weighted w_p w_q
                double ts = 0.0, tm = 0.0, ms = 0.0, mm = 0.0;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (4 * r >= NP) continue;
                    const double ys = out_s ? wj[r] * (double)T(ds[r]) : 0.0;
                    const double ym = out_m ? wj[r] * (double)T(dm[r]) : 0.0;
                    ts += ys;
                    ms += fabs(ys);
                    tm += ym;
                    mm += fabs(ym);
                }
                double *q = acc + tid;
                q[(4 * v + 0) * C::NT] += wpp * ts;
                q[(4 * v + 1) * C::NT] += wpp * ms;
                q[(4 * v + 2) * C::NT] += wpp * tm;
                q[(4 * v + 3) * C::NT] += wpp * mm;
            }
            // every lane stores (no branch: a branch around a store leaves the compiler
            // unsure how many memory operations are outstanding, and it then waits for all
            // of them before the next); masked lanes get an offset beyond the array
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                if (4 * r >= NP) continue;                 // no face node in any lane
                const int j = rd_node(kq, r);
                const uint32_t jj = (uint32_t)min(j, NP - 1);
                const uint32_t o_s = ((line + jj) * (uint32_t)a.nfs + (uint32_t)oc_s) * (uint32_t)sizeof(T) +
                                     (uint32_t)v * (uint32_t)pbytes_s;
                const uint32_t o_m = ((line + jj) * (uint32_t)a.nfm + (uint32_t)oc_m) * (uint32_t)sizeof(T) +
                                     (uint32_t)v * (uint32_t)pbytes_m;
                buf_store<T>(T(ds[r]), rF_s, out_s && j < NP ? o_s : kRdOff, 0);
                buf_store<T>(T(dm[r]), rF_m, out_m && j < NP ? o_m : kRdOff, 0);
            }
        }
    }
    if constexpr (FUSE) {
        // the workgroup's partials: 16 chunks of NT / 16 lanes per slot, then the chunks,
        // in fixed orders; partial g = 2 v + side at a.cons[(g * gridDim.x + block) * 2 + m].
        // Chunk c of a slot holds lanes c, c + 16, c + 32, ..: the chunks of a slot read 16
        // consecutive doubles at a time (with a contiguous run of lanes per chunk, every
        // lane of a wave read the same LDS bank pair)
        constexpr int CH = C::NT / 16;
        __syncthreads();
        for (int t = tid; t < 320; t += C::NT) {
            const int k = t >> 4, c = t & 15;
            const double *q = acc + k * C::NT + c;
            double x = 0.0;
            for (int l = 0; l < CH; ++l) x += q[16 * l];
            red[t] = x;
        }
        __syncthreads();
        if (tid < 20 && a.cons) {
            double x = 0.0;
            for (int c = 0; c < 16; ++c) x += red[tid * 16 + c];
            a.cons[((size_t)(tid >> 1) * gridDim.x + blockIdx.x) * 2 + (tid & 1)] = x;
        }
        __syncthreads();
    }
    return Cursor::next_rot(a.n_tiles, C::WAVES, rot);
}

// The BR1 lifting surface term through the register-direct body: four free waves per
// workgroup below NP = 8, the eight-wave lockstep rounds of the flux launches from NP = 8.
template <typename T, int NP, bool MET>
__global__ __launch_bounds__(64 * rd_lift_waves(NP)) void k_mortar_lift_rd(FluxArgs<T> a)
{
    __shared__ double work[assemble_scratch<NP>()];
    __shared__ T mats[8 * NP * NP];
    __shared__ double wq[NP];
    __shared__ double acc[1];
    __shared__ double red[1];
    rd_interface<T, NP, false, MET, 0, 0, rd_lift_waves(NP), true>(a, work, mats, wq, acc, red);
}

template <typename T, int NP, bool NSV, bool MET, int RIEM, int PREC>
__global__ __launch_bounds__(64 * rd_waves((int)sizeof(T), NSV, NP)) void k_mortar_flux_rd(FluxArgs<T> a)
{
    constexpr int WV = rd_waves((int)sizeof(T), NSV, NP);
    constexpr int NT = 64 * WV;
    __shared__ double work[assemble_scratch<NP>()];
    __shared__ T mats[8 * NP * NP];          // Pf[4][NP][NP], Pb[4][NP][NP]
    __shared__ double wq[NP];
    constexpr bool FUSE = sizeof(T) == 4;
    __shared__ double acc[FUSE ? 20 * NT : 1];
    __shared__ double red[FUSE ? 320 : 1];
    rd_interface<T, NP, NSV, MET, RIEM, PREC, WV>(a, work, mats, wq, acc, red);
}

// Every interface of a batch in one persistent launch (degrees N = 3, 5, 7, element type
// FP32): the workgroups take the interfaces one after the other, each with its own
// XCD-aware wave cursor.  Each interface starts the order of its workgroups after those
// that took the previous interface's last, partial round, so that no workgroup takes
// the partial round of every interface.  The bodies are inlined; the host launches this
// kernel only for batches whose degrees are all in {3, 5, 7}.
template <bool NSV, int RIEM>
__global__ __launch_bounds__(64 * kRdBatchWaves) __attribute__((amdgpu_waves_per_eu(2))) void k_mortar_flux_rd_batch(BatchArgs<float> b)
{
    constexpr int NPM = 8;
    constexpr int NT = 64 * kRdBatchWaves;
    __shared__ double work[assemble_scratch<NPM>()];
    __shared__ float mats[8 * NPM * NPM];
    __shared__ double wq[NPM];
    __shared__ double acc[20 * NT];
    __shared__ double red[320];
    int rot = 0;
    for (int i = 0; i < b.n_if; ++i) {
        const bool met = b.met[i] != 0;
#define MORTAR_RD_BATCH_NP(NPV)                                                               \
    if (b.np[i] == NPV) {                                                                     \
        rot = met ? rd_interface<float, NPV, NSV, true, RIEM, 0, kRdBatchWaves>(b.a[i], work, mats, wq, acc, red, rot) \
                  : rd_interface<float, NPV, NSV, false, RIEM, 0, kRdBatchWaves>(b.a[i], work, mats, wq, acc, red, rot); \
        continue;                                                                             \
    }
        MORTAR_RD_BATCH_NP(4) MORTAR_RD_BATCH_NP(6) MORTAR_RD_BATCH_NP(8)
#undef MORTAR_RD_BATCH_NP
    }
}

}  // namespace mortar

// ---- launch helpers shared by the instantiation units --------------------------------
namespace mortar {

template <typename T, int NP, bool NSV, bool MET, int RIEM, int PREC>
static hipError_t rd_go(const FluxArgs<T> &a, int grid, hipStream_t st)
{
    hipLaunchKernelGGL((k_mortar_flux_rd<T, NP, NSV, MET, RIEM, PREC>), dim3(grid), dim3(64 * rd_waves((int)sizeof(T), NSV, NP)), 0,
                       st, a);
    return hipGetLastError();
}

template <typename T, int NP, bool NSV, bool MET, int RIEM, int PREC>
static int rd_occ1()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, reinterpret_cast<const void *>(&k_mortar_flux_rd<T, NP, NSV, MET, RIEM, PREC>), 64 * rd_waves((int)sizeof(T), NSV, NP),
            0) != hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

// Dispatch over (physics, metrics, Riemann solver) for one degree and precision mode.
template <typename T, int NP, int PREC>
static hipError_t rd_pick(const FluxArgs<T> &a, int grid, bool ns, bool met, int riem,
                          hipStream_t st)
{
    if (ns) {
        if (met) return riem ? rd_go<T, NP, true, true, 1, PREC>(a, grid, st)
                             : rd_go<T, NP, true, true, 0, PREC>(a, grid, st);
        return riem ? rd_go<T, NP, true, false, 1, PREC>(a, grid, st)
                    : rd_go<T, NP, true, false, 0, PREC>(a, grid, st);
    }
    if (met) return riem ? rd_go<T, NP, false, true, 1, PREC>(a, grid, st)
                         : rd_go<T, NP, false, true, 0, PREC>(a, grid, st);
    return riem ? rd_go<T, NP, false, false, 1, PREC>(a, grid, st)
                : rd_go<T, NP, false, false, 0, PREC>(a, grid, st);
}

template <typename T, int NP>
static hipError_t rd_lift_go(const FluxArgs<T> &a, int grid, bool met, hipStream_t st)
{
    if (met) hipLaunchKernelGGL((k_mortar_lift_rd<T, NP, true>), dim3(grid), dim3(64 * rd_lift_waves(NP)), 0, st, a);
    else hipLaunchKernelGGL((k_mortar_lift_rd<T, NP, false>), dim3(grid), dim3(64 * rd_lift_waves(NP)), 0, st, a);
    return hipGetLastError();
}

template <typename T, int NP>
static int rd_lift_occ(bool met)
{
    int nb = 0;
    const void *k = met ? reinterpret_cast<const void *>(&k_mortar_lift_rd<T, NP, true>)
                        : reinterpret_cast<const void *>(&k_mortar_lift_rd<T, NP, false>);
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, 64 * rd_lift_waves(NP), 0) != hipSuccess) return 1;
    return nb > 0 ? nb : 1;
}

template <typename T, int NP, int PREC>
static int rd_occ(bool ns, bool met, int riem)
{
    if (ns) {
        if (met) return riem ? rd_occ1<T, NP, true, true, 1, PREC>() : rd_occ1<T, NP, true, true, 0, PREC>();
        return riem ? rd_occ1<T, NP, true, false, 1, PREC>() : rd_occ1<T, NP, true, false, 0, PREC>();
    }
    if (met) return riem ? rd_occ1<T, NP, false, true, 1, PREC>() : rd_occ1<T, NP, false, true, 0, PREC>();
    return riem ? rd_occ1<T, NP, false, false, 1, PREC>() : rd_occ1<T, NP, false, false, 0, PREC>();
}

}  // namespace mortar

#define MORTAR_RD_NP_SWITCH(EXPR, DEFAULT)                                              \
    switch (NP) {                                                                       \
    case 2: return EXPR(2); case 3: return EXPR(3); case 4: return EXPR(4);            \
    case 5: return EXPR(5); case 6: return EXPR(6); case 7: return EXPR(7);            \
    case 8: return EXPR(8); case 9: return EXPR(9); case 10: return EXPR(10);          \
    default: return DEFAULT;                                                            \
    }
