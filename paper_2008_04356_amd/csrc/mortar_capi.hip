// C ABI of the mortar library (declared in include/mortar.h): descriptor validation,
// FP64 basis constants, device buffers, per-stage updates and kernel dispatch.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <cstdio>
#include <cstdlib>
#include <new>
#include <string>
#include <vector>

#include "k_flux.h"
#include "mortar_internal.h"

namespace mortar {
hipError_t launch_flux_f32(const FluxArgs<float> &a, int NP, int grid, bool ns, bool met,
                           int riem, hipStream_t st);
hipError_t launch_flux_f64(const FluxArgs<double> &a, int NP, int grid, bool ns, bool met,
                           int riem, hipStream_t st);
int flux_tile_capacity_f32(int NP, bool ns, bool met);
int flux_tile_capacity_f64(int NP, bool ns, bool met);
int flux_occupancy_f32(int NP, bool ns, bool met, int riem);
int flux_wide_occupancy_f32(int NP, bool ns, bool met, int riem);
int flux_wide_tile_capacity_f32(int NP, bool ns, bool met);
hipError_t launch_flux_wide_f32(const FluxArgs<float> &a, int NP, int grid, bool ns, bool met,
                                int riem, hipStream_t st);
int flux_occupancy_f64(int NP, bool ns, bool met, int riem);
int flux_hyb_occupancy_f32(int NP, bool ns, bool met, int riem);
int lift_occupancy(int NP, bool met, bool f64);
int lift_tile_capacity(int NP, bool met, bool f64);
hipError_t launch_lift_f32(const FluxArgs<float> &a, int NP, int grid, bool met, hipStream_t st);
int lift_rd_occupancy_f32(int NP, bool met);
hipError_t launch_lift_rd_f32(const FluxArgs<float> &a, int NP, int grid, bool met, hipStream_t st);
hipError_t launch_lift_f64(const FluxArgs<double> &a, int NP, int grid, bool met, hipStream_t st);
int flux_hyb_tile_capacity_f32(int NP, bool ns, bool met);
hipError_t launch_flux_hyb_f32(const FluxArgs<float> &a, int NP, int grid, bool ns, bool met,
                               int riem, hipStream_t st);
int flux_mfma_occupancy_f32(int NP, bool ns, bool met, int riem);
int flux_mfma_occupancy_f64(int NP, bool ns, bool met, int riem);
hipError_t launch_flux_mfma_f32(const FluxArgs<float> &a, int NP, int grid, bool ns, bool met,
                                int riem, hipStream_t st);
hipError_t launch_flux_mfma_f64(const FluxArgs<double> &a, int NP, int grid, bool ns, bool met,
                                int riem, hipStream_t st);
hipError_t launch_flux_batch_f32(const BatchArgs<float> &b, int grid, bool ns, int riem,
                                 bool turbine, hipStream_t st);
hipError_t launch_flux_batch_f64(const BatchArgs<double> &b, int grid, bool ns, int riem,
                                 bool turbine, hipStream_t st);
int flux_batch_occupancy_f32(bool ns, int riem, bool turbine);
int flux_rd_batch_occupancy_f32(bool ns, int riem);
hipError_t launch_flux_rd_batch_f32(const BatchArgs<float> &b, int grid, bool ns, int riem,
                                    hipStream_t st);
int flux_rd_occupancy_f32(int NP, bool ns, bool met, int riem);
// the conservation kernels' host handles (k_topology.hip)
bool is_conservation_kernel(const void *func);
int flux_rd_occupancy_f64(int NP, bool ns, bool met, int riem);
int flux_rd_occupancy_bf16(int NP, bool ns, bool met, int riem);

int flux_rd_occupancy_fp16(int NP, bool ns, bool met, int riem);
hipError_t launch_flux_rd_f32(const FluxArgs<float> &a, int NP, int grid, bool ns, bool met,
                              int riem, hipStream_t st);
hipError_t launch_flux_rd_f64(const FluxArgs<double> &a, int NP, int grid, bool ns, bool met,
                              int riem, hipStream_t st);
hipError_t launch_flux_rd_bf16(const FluxArgs<float> &a, int NP, int grid, bool ns, bool met,
                               int riem, hipStream_t st);
hipError_t launch_flux_rd_fp16(const FluxArgs<float> &a, int NP, int grid, bool ns, bool met,
                               int riem, hipStream_t st);
int flux_batch_occupancy_f64(bool ns, int riem, bool turbine);

// ------------------------------------------------------------------------------------
// FP64 node sets by bracketing and bisection (roots of P_NP for Gauss, of P_N' for
// Gauss-Lobatto), weights from the Legendre polynomials.
// ------------------------------------------------------------------------------------

// Legendre P_k(x) for k = n and n - 1 by the three-term recurrence.
static void legendre_pair(int n, double x, double &pn, double &pn1)
{
    double a = 1.0, b = x;  // P_0, P_1
    if (n == 0) { pn = 1.0; pn1 = 0.0; return; }
    for (int k = 2; k <= n; ++k) {
        const double c = ((2 * k - 1) * x * b - (k - 1) * a) / k;
        a = b;
        b = c;
    }
    pn = b;
    pn1 = a;
}

// (1 - x^2) P_n'(x) = n (P_{n-1} - x P_n): sign-equivalent to P_n' inside (-1, 1).
static double dlegendre_scaled(int n, double x)
{
    double pn, pn1;
    legendre_pair(n, x, pn, pn1);
    return n * (pn1 - x * pn);
}

template <typename Fn>
static std::vector<double> interior_roots(Fn f, int count)
{
    // Sign changes on a uniform grid bracket the simple roots; a root that falls exactly
    // on a grid point is taken as is and not bracketed again from its right.
    std::vector<double> roots;
    const int M = 4000;
    const double lo0 = -1.0 + 1e-12, span = 2.0 - 2e-12;
    double xa = lo0, fa = f(xa);
    for (int i = 1; i <= M && (int)roots.size() < count; ++i) {
        const double xb = lo0 + span * i / M, fb = f(xb);
        if (fb == 0.0) {
            roots.push_back(xb);
        } else if (fa != 0.0 && ((fa < 0.0) != (fb < 0.0))) {
            double lo = xa, hi = xb, flo = fa;
            for (int it = 0; it < 200; ++it) {
                const double mid = 0.5 * (lo + hi);
                if (mid == lo || mid == hi) break;
                const double fm = f(mid);
                if (fm == 0.0) { lo = hi = mid; break; }
                if ((fm < 0.0) == (flo < 0.0)) { lo = mid; flo = fm; } else hi = mid;
            }
            roots.push_back(0.5 * (lo + hi));
        }
        xa = xb;
        fa = fb;
    }
    return roots;
}

static bool gauss_nodes(int np, double *x, double *w)
{
    auto f = [np](double t) { double a, b; legendre_pair(np, t, a, b); return a; };
    std::vector<double> r = interior_roots(f, np);
    if ((int)r.size() != np) return false;
    for (int i = 0; i < np; ++i) {
        x[i] = r[i];
        // w = 2 / ((1 - x^2) P_n'(x)^2) with P_n' = n (P_{n-1} - x P_n) / (1 - x^2); the
        // x P_n term (P_n is only zero up to rounding at the computed root) keeps the
        // weights accurate to a few ulps at the higher degrees
        double pn, pn1;
        legendre_pair(np, r[i], pn, pn1);
        const double omx2 = (1.0 - r[i]) * (1.0 + r[i]);
        const double dp = np * (pn1 - r[i] * pn) / omx2;
        w[i] = 2.0 / (omx2 * dp * dp);
    }
    return true;
}

static bool lobatto_nodes(int N, double *x, double *w)
{
    auto f = [N](double t) { return dlegendre_scaled(N, t); };
    std::vector<double> r = interior_roots(f, N - 1);
    if ((int)r.size() != N - 1) return false;
    x[0] = -1.0;
    x[N] = 1.0;
    for (int i = 0; i < N - 1; ++i) x[i + 1] = r[i];
    for (int i = 0; i <= N; ++i) {
        double pn, pn1;
        legendre_pair(N, x[i], pn, pn1);
        w[i] = 2.0 / (N * (N + 1.0) * pn * pn);
    }
    return true;
}

static double lagrange_bary(int np, const double *x, const double *bw, int j, double t)
{
    for (int m = 0; m < np; ++m)
        if (t == x[m]) return m == j ? 1.0 : 0.0;
    double den = 0.0;
    for (int m = 0; m < np; ++m) den += bw[m] / (t - x[m]);
    return bw[j] / (t - x[j]) / den;
}

static bool invert_gj(int n, const double *A, double *R, int ld)
{
    double a[kMaxNP][2 * kMaxNP];
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            a[i][j] = A[i * n + j];
            a[i][n + j] = i == j;
        }
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(a[r][c]) > std::fabs(a[p][c])) p = r;
        if (a[p][c] == 0.0) return false;
        for (int j = 0; j < 2 * n; ++j) std::swap(a[c][j], a[p][j]);
        const double d = 1.0 / a[c][c];
        for (int j = 0; j < 2 * n; ++j) a[c][j] *= d;
        for (int r = 0; r < n; ++r)
            if (r != c) {
                const double g = a[r][c];
                for (int j = 0; j < 2 * n; ++j) a[r][j] -= g * a[c][j];
            }
    }
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) R[i * ld + j] = a[i][n + j];
    return true;
}

static bool basis_consts(int N, int node_set, BasisConsts &c)
{
    std::memset(&c, 0, sizeof(c));
    const int np = N + 1;
    const bool ok = node_set == MORTAR_NODES_GAUSS ? gauss_nodes(np, c.x, c.w)
                                                   : lobatto_nodes(N, c.x, c.w);
    if (!ok || !gauss_nodes(np, c.t, c.tw)) return false;
    for (int j = 0; j < np; ++j) {
        double p = 1.0;
        for (int m = 0; m < np; ++m)
            if (m != j) p *= c.x[j] - c.x[m];
        c.bw[j] = 1.0 / p;
    }
    for (int r = 0; r < np; ++r)
        for (int q = 0; q < np; ++q) c.Lt[r * kMaxNP + q] = lagrange_bary(np, c.x, c.bw, q, c.t[r]);
    // mass matrix M_ij = int l_i l_j with the np-point Gauss rule (exact to degree 2N+1)
    double M[kMaxNP * kMaxNP];
    for (int i = 0; i < np; ++i)
        for (int j = 0; j < np; ++j) {
            double acc = 0.0;
            for (int r = 0; r < np; ++r) acc += c.tw[r] * c.Lt[r * kMaxNP + i] * c.Lt[r * kMaxNP + j];
            M[i * np + j] = acc;
        }
    return invert_gj(np, M, c.Minv, kMaxNP);
}

// ------------------------------------------------------------------------------------

// The register-direct kernel addresses every input and output array with 32-bit byte
// offsets: each array must stay at most kRdMaxBytes (just below 4 GiB).
static bool rd_addressable(const mortar_iface_desc &d)
{
    const int64_t P = (int64_t)(d.N + 1) * (d.N + 1);
    const int64_t elem = d.precision == MORTAR_FP64 ? 8 : 4;
    const int64_t vars = d.physics == MORTAR_NAVIER_STOKES ? 15 : 5;
    const int64_t nf = std::max<int64_t>(d.n_face_static, d.n_face_moving);
    return vars * P * nf * elem <= kRdMaxBytes;
}

// The VALU-projection kernels store through buffer descriptors over one side's five
// flux planes and mask lanes with an offset of 2 GiB: each flux array must stay below it.
static bool valu_addressable(const mortar_iface_desc &d)
{
    const int64_t P = (int64_t)(d.N + 1) * (d.N + 1);
    const int64_t elem = d.precision == MORTAR_FP64 ? 8 : 4;
    const int64_t nf = std::max<int64_t>(d.n_face_static, d.n_face_moving);
    return 5 * P * nf * elem < ((int64_t)1 << 31);
}

static int validate_one(const mortar_iface_desc &d)
{
    if (d.N < 1 || d.n_par < 1 || d.n_perp < 1) return MORTAR_ERR_INVALID_ARG;
    if (d.N > kMaxN) return MORTAR_ERR_UNSUPPORTED;
    if (d.node_set != MORTAR_NODES_GAUSS && d.node_set != MORTAR_NODES_LGL)
        return MORTAR_ERR_INVALID_ARG;
    if (d.physics != MORTAR_EULER && d.physics != MORTAR_NAVIER_STOKES) return MORTAR_ERR_INVALID_ARG;
    if (d.riemann != MORTAR_FLUX_LF && d.riemann != MORTAR_FLUX_ROE) return MORTAR_ERR_INVALID_ARG;
    if (d.precision < MORTAR_FP64 || d.precision > MORTAR_FP16_MFMA) return MORTAR_ERR_INVALID_ARG;
    if ((d.precision == MORTAR_BF16_MFMA || d.precision == MORTAR_FP16_MFMA) &&
        (!rd_addressable(d) || d.N > kMaxNFast))
        return MORTAR_ERR_UNSUPPORTED;
    // above kMaxNFast only the VALU-projection kernel exists: its flux arrays must stay
    // below 2 GiB
    if (d.N > kMaxNFast && !valu_addressable(d)) return MORTAR_ERR_UNSUPPORTED;
    const int64_t F = (int64_t)d.n_par * d.n_perp;
    if (F > (int64_t)1 << 28) return MORTAR_ERR_UNSUPPORTED;
    if (d.n_face_static < F || d.n_face_moving < F) return MORTAR_ERR_INVALID_ARG;
    const int64_t P = (int64_t)(d.N + 1) * (d.N + 1);
    if (P * 20 * (int64_t)std::max(d.n_face_static, d.n_face_moving) > ((int64_t)1 << 40))
        return MORTAR_ERR_UNSUPPORTED;
    if (!d.face_id_static || !d.face_id_moving) return MORTAR_ERR_INVALID_ARG;
    if (!(std::isfinite(d.l_par) && d.l_par > 0.0)) return MORTAR_ERR_INVALID_ARG;
    if (!(std::isfinite(d.gamma) && d.gamma > 1.0)) return MORTAR_ERR_INVALID_ARG;
    if (d.physics == MORTAR_NAVIER_STOKES &&
        !(std::isfinite(d.mu) && d.mu >= 0.0 && std::isfinite(d.Pr) && d.Pr > 0.0))
        return MORTAR_ERR_INVALID_ARG;
    if (!d.metrics) {
        const double nn = d.normal[0] * d.normal[0] + d.normal[1] * d.normal[1] +
                          d.normal[2] * d.normal[2];
        if (!(std::isfinite(nn) && std::fabs(nn - 1.0) < 1e-6 && std::isfinite(d.dS)))
            return MORTAR_ERR_INVALID_ARG;
    }
    // face ids: in range and distinct per side
    for (int side = 0; side < 2; ++side) {
        const int32_t *fid = side ? d.face_id_moving : d.face_id_static;
        const int nf = side ? d.n_face_moving : d.n_face_static;
        std::vector<char> seen(nf, 0);
        for (int64_t i = 0; i < F; ++i) {
            const int32_t c = fid[i];
            if (c < 0 || c >= nf || seen[c]) return MORTAR_ERR_INVALID_ARG;
            seen[c] = 1;
        }
        const int32_t *own = side ? d.owner_moving : d.owner_static;
        if (own) {
            std::vector<int32_t> u(own, own + F);
            std::sort(u.begin(), u.end());
            if (std::unique(u.begin(), u.end()) - u.begin() > kMaxOwners) return MORTAR_ERR_UNSUPPORTED;
        }
    }
    return MORTAR_OK;
}

static void free_iface(Iface &f)
{
    void *bufs[] = {f.d_fid_s, f.d_fid_m, f.d_oid_s, f.d_oid_m, f.d_oval_s, f.d_oval_m,
                    f.d_metrics, f.d_params, f.d_basis, f.d_A[0], f.d_A[1], f.d_m[0],
                    f.d_m[1], f.d_hist, f.d_pair, f.d_cons, f.d_cons_out, f.d_cons_wg};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    f = Iface();
}

#define TRY_HIP(x)                                   \
    do {                                             \
        if ((x) != hipSuccess) return MORTAR_ERR_HIP; \
    } while (0)

template <typename T>
static int upload(T **dst, const T *src, size_t count)
{
    if (hipMalloc((void **)dst, sizeof(T) * std::max<size_t>(count, 1)) != hipSuccess)
        return MORTAR_ERR_OOM;
    if (count) TRY_HIP(hipMemcpy(*dst, src, sizeof(T) * count, hipMemcpyHostToDevice));
    return MORTAR_OK;
}

// Dense owner ids (ascending owner value) of one side.
static void owner_ids(const int32_t *own, int64_t F, std::vector<int32_t> &ids,
                      std::vector<int32_t> &vals)
{
    ids.assign(F, 0);
    vals.assign(1, 0);
    if (!own) return;
    vals.assign(own, own + F);
    std::sort(vals.begin(), vals.end());
    vals.erase(std::unique(vals.begin(), vals.end()), vals.end());
    for (int64_t i = 0; i < F; ++i)
        ids[i] = (int32_t)(std::lower_bound(vals.begin(), vals.end(), own[i]) - vals.begin());
}

// Resident workgroups per CU of a kernel variant for this interface.
static int variant_occupancy(const Iface &f, int variant)
{
    const bool ns = f.d.physics == MORTAR_NAVIER_STOKES, met = f.d_metrics != nullptr;
    const int riem = f.d.riemann == MORTAR_FLUX_ROE;
    if (variant == 0)
        return f.elem == 8 ? flux_occupancy_f64(f.NP, ns, met, riem) : flux_occupancy_f32(f.NP, ns, met, riem);
    if (variant == 1)
        return f.elem == 8 ? flux_mfma_occupancy_f64(f.NP, ns, met, riem)
                           : flux_mfma_occupancy_f32(f.NP, ns, met, riem);
    if (variant == 3) return flux_wide_occupancy_f32(f.NP, ns, met, riem);
    if (variant == 4) return flux_hyb_occupancy_f32(f.NP, ns, met, riem);
    if (f.lp == 1) return flux_rd_occupancy_bf16(f.NP, ns, met, riem);
    if (f.lp == 2) return flux_rd_occupancy_fp16(f.NP, ns, met, riem);
    return f.elem == 8 ? flux_rd_occupancy_f64(f.NP, ns, met, riem) : flux_rd_occupancy_f32(f.NP, ns, met, riem);
}

static bool variant_allowed(const Iface &f, int variant)
{
    if (variant < 0 || variant > 4) return false;
    if (f.d.N > kMaxNFast) return variant == 0 && valu_addressable(f.d);
    if (f.lp) return variant == 2;
    if (variant == 4)
        return f.elem == 4 && valu_addressable(f.d) &&
               flux_hyb_tile_capacity_f32(f.NP, f.d.physics == MORTAR_NAVIER_STOKES, f.d_metrics != nullptr) > 0;
    if (variant == 0 || variant == 3) return valu_addressable(f.d) && (variant == 0 || f.elem == 4);
    return variant != 2 || rd_addressable(f.d);
}

static int setup_one(const mortar_iface_desc &d, Iface &f)
{
    f.d = d;
    f.d.face_id_static = f.d.face_id_moving = nullptr;
    f.d.owner_static = f.d.owner_moving = nullptr;
    f.d.metrics = nullptr;
    f.NP = d.N + 1;
    f.P = f.NP * f.NP;
    f.F = d.n_par * d.n_perp;
    f.elem = d.precision == MORTAR_FP64 ? 8 : 4;
    int rc;
    if ((rc = upload(&f.d_fid_s, d.face_id_static, f.F))) return rc;
    if ((rc = upload(&f.d_fid_m, d.face_id_moving, f.F))) return rc;
    std::vector<int32_t> ids, vals;
    owner_ids(d.owner_static, f.F, ids, vals);
    f.R_s = (int)vals.size();
    if ((rc = upload(&f.d_oid_s, ids.data(), ids.size()))) return rc;
    if ((rc = upload(&f.d_oval_s, vals.data(), vals.size()))) return rc;
    owner_ids(d.owner_moving, f.F, ids, vals);
    f.R_m = (int)vals.size();
    if ((rc = upload(&f.d_oid_m, ids.data(), ids.size()))) return rc;
    if ((rc = upload(&f.d_oval_m, vals.data(), vals.size()))) return rc;
    if (d.metrics) {
        const size_t cnt = (size_t)4 * f.P * d.n_face_static;
        if (f.elem == 8) {
            double *p;
            if ((rc = upload(&p, d.metrics, cnt))) return rc;
            f.d_metrics = p;
        } else {
            std::vector<float> tmp(d.metrics, d.metrics + cnt);
            float *p;
            if ((rc = upload(&p, tmp.data(), cnt))) return rc;
            f.d_metrics = p;
        }
    }
    BasisConsts bc;
    if (!basis_consts(d.N, d.node_set, bc)) return MORTAR_ERR_UNSUPPORTED;
    if ((rc = upload(&f.d_basis, &bc, 1))) return rc;
    if (hipMalloc((void **)&f.d_params, param_bytes(f.NP)) != hipSuccess) return MORTAR_ERR_OOM;
    TRY_HIP(hipMemset(f.d_params, 0, param_bytes(f.NP)));
    for (int s = 0; s < 2; ++s) {
        const int nf = s ? d.n_face_moving : d.n_face_static;
        if (hipMalloc((void **)&f.d_A[s], sizeof(int32_t) * 5 * 2 * (size_t)f.F) != hipSuccess ||
            hipMalloc((void **)&f.d_m[s], sizeof(int32_t) * 2 * (size_t)nf) != hipSuccess)
            return MORTAR_ERR_OOM;
    }
    if (hipMalloc((void **)&f.d_pair, sizeof(int32_t) * 2 * (size_t)d.n_par) != hipSuccess)
        return MORTAR_ERR_OOM;
    f.n_sort_blocks = (2 * f.F + kSortBlock - 1) / kSortBlock;
    const int R = std::max(f.R_s, f.R_m);
    if (hipMalloc((void **)&f.d_hist, sizeof(int32_t) * (size_t)R * f.n_sort_blocks) != hipSuccess)
        return MORTAR_ERR_OOM;
    {
        const bool ns = d.physics == MORTAR_NAVIER_STOKES, met = d.metrics != nullptr;
        const int riem = d.riemann == MORTAR_FLUX_ROE;
        // kernel variant: the low-precision GEMM modes exist only in the register-direct
        // kernel; otherwise MORTAR_FLUX_KERNEL = valu | mfma | rd selects one
        const char *kv = std::getenv("MORTAR_FLUX_KERNEL");
        const std::string kname = kv ? kv : "";
        f.lp = d.precision == MORTAR_BF16_MFMA ? 1 : (d.precision == MORTAR_FP16_MFMA ? 2 : 0);
        f.flux_variant = kname == "mfma" ? 1 : kname == "rd" ? 2 : kname == "hyb" ? 4 : 0;
        if (f.lp) f.flux_variant = 2;
        if (!variant_allowed(f, f.flux_variant)) f.flux_variant = 0;
        if (!variant_allowed(f, f.flux_variant)) f.flux_variant = 1;   // MFMA-LDS: any size
        f.flux_occ = variant_occupancy(f, f.flux_variant);
        (void)ns; (void)met; (void)riem;
    }
    f.n_cons_blocks = cons_blocks(f.P, f.F);
    if (hipMalloc((void **)&f.d_cons_out, sizeof(double) * 15) != hipSuccess) return MORTAR_ERR_OOM;
    if (hipMalloc((void **)&f.d_cons, sizeof(double) * 40 * (size_t)f.n_cons_blocks) != hipSuccess)
        return MORTAR_ERR_OOM;
    if (hipMalloc((void **)&f.d_cons_wg, sizeof(double) * 20 * (size_t)kConsGridMax) != hipSuccess)
        return MORTAR_ERR_OOM;
    return MORTAR_OK;
}

// Displacement split (Sec. 4.3): n = floor(delta / l), s = the rest in [0, 1), in FP64.
static void decompose(double delta, double l, int64_t &n, double &s)
{
    const double q = delta / l;
    const double fl = std::floor(q);
    double frac = q - fl;
    int64_t k = (int64_t)fl;
    if (frac >= 1.0) {
        frac -= 1.0;
        k += 1;
    }
    if (!(frac > 0.0)) frac = 0.0;
    n = k;
    s = frac;
}

// Conservation sums of a face-flux pair: from the partials of the fused flux launch
// when these are its outputs (the sums of exactly the values it wrote), else by a pass
// over the arrays.
static hipError_t launch_conservation_any(const Iface &f, const void *Fs, const void *Fm, double *d_out,
                                          hipStream_t st)
{
    if (f.cons_nb > 0 && f.cons_Fs == Fs && f.cons_Fm == Fm) return launch_conservation_final(f, d_out, st);
    return launch_conservation(f, Fs, Fm, d_out, st);
}

static int apply_update(Handle *h, const int64_t *n, const double *s, hipStream_t st)
{
    for (auto &f : h->ifs) {
        const size_t i = &f - h->ifs.data();
        f.n = n[i];
        f.s = s[i];
        const int64_t np = f.d.n_par;
        const int64_t nmod = ((f.n % np) + np) % np;
        if (nmod != f.nmod_built) {
            TRY_HIP(launch_index_map(f, 0, st));
            TRY_HIP(launch_index_map(f, 1, st));
            f.nmod_built = nmod;
        }
        f.ready = true;
    }
    return MORTAR_OK;
}

}  // namespace mortar

namespace mortar {
template <typename T>
void fill_args(const Iface &f, const void *Us, const void *Um, const void *Gs, const void *Gm,
               void *Fs, void *Fm, FluxArgs<T> &a, int &n_tiles);
static int tiled_grid(const Iface &f, int n_cu, int nt);
static int rd_grid_of(const Iface &f, int n_cu, int nt);
static int rd_batch_grid(const Handle &h, int total);
template <typename T>
static void set_cons(const Iface &f, FluxArgs<T> &a, int grid, const void *Fs, const void *Fm);
}  // namespace mortar

using namespace mortar;

struct mortar_handle : public mortar::Handle {};

// A captured stage: the flux launch(es) of a handle for fixed buffers (and, from
// mortar_graph_create_cons, the stage's conservation sums).
struct mortar_graph {
    mortar_handle *h = nullptr;
    unsigned epoch = 0;                      // tuning epoch of the handle at capture
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<hipGraphNode_t> nodes;       // flux kernel nodes in launch order
    std::vector<const void *> Us, Um, Gs, Gm;
    std::vector<void *> Fs, Fm;
};

extern "C" {

const char *mortar_error_string(int code)
{
    switch (code) {
    case MORTAR_OK: return "ok";
    case MORTAR_ERR_INVALID_ARG: return "invalid argument";
    case MORTAR_ERR_UNSUPPORTED: return "unsupported configuration";
    case MORTAR_ERR_OOM: return "out of memory";
    case MORTAR_ERR_HIP: return "HIP runtime error";
    case MORTAR_ERR_NOT_READY: return "no displacement set yet";
    default: return "unknown error";
    }
}

int mortar_validate(const mortar_iface_desc *desc, int n_iface)
{
    if (!desc || n_iface < 1) return MORTAR_ERR_INVALID_ARG;
    for (int i = 0; i < n_iface; ++i) {
        const int rc = validate_one(desc[i]);
        if (rc) return rc;
    }
    return MORTAR_OK;
}

int mortar_basis(int N, int node_set, double *x, double *w)
{
    if (!x || !w || N < 1) return MORTAR_ERR_INVALID_ARG;
    if (N > kMaxN) return MORTAR_ERR_UNSUPPORTED;
    if (node_set != MORTAR_NODES_GAUSS && node_set != MORTAR_NODES_LGL) return MORTAR_ERR_INVALID_ARG;
    BasisConsts c;
    if (!basis_consts(N, node_set, c)) return MORTAR_ERR_UNSUPPORTED;
    for (int i = 0; i <= N; ++i) {
        x[i] = c.x[i];
        w[i] = c.w[i];
    }
    return MORTAR_OK;
}

int mortar_decompose_displacement(double delta, double l_par, int64_t *n, double *s)
{
    if (!n || !s || !std::isfinite(delta) || !(std::isfinite(l_par) && l_par > 0.0))
        return MORTAR_ERR_INVALID_ARG;
    const double q = delta / l_par;
    if (!(std::fabs(q) < 9.0e15)) return MORTAR_ERR_INVALID_ARG;
    decompose(delta, l_par, *n, *s);
    return MORTAR_OK;
}

int mortar_setup(const mortar_iface_desc *desc, int n_iface, mortar_handle **out)
{
    if (!out) return MORTAR_ERR_INVALID_ARG;
    int rc = mortar_validate(desc, n_iface);
    if (rc) return rc;
    mortar_handle *h = new (std::nothrow) mortar_handle();
    if (!h) return MORTAR_ERR_OOM;
    if (hipGetDevice(&h->device) != hipSuccess ||
        hipDeviceGetAttribute(&h->n_cu, hipDeviceAttributeMultiprocessorCount, h->device) !=
            hipSuccess) {
        delete h;
        return MORTAR_ERR_HIP;
    }
    // the static partials array of mortar_conservation_device_noalloc: its address on
    // this device, looked up once per device while the device is current
    if (static_cons_scratch(h->device, &h->static_scratch) != hipSuccess) {
        delete h;
        return MORTAR_ERR_HIP;
    }
    h->ifs.resize(n_iface);
    for (int i = 0; i < n_iface; ++i) {
        rc = setup_one(desc[i], h->ifs[i]);
        if (rc) {
            for (auto &f : h->ifs) free_iface(f);
            delete h;
            return rc;
        }
    }
    // One persistent launch for every interface when they share element type, physics and
    // flux (and use the VALU-projection kernel).
    if (n_iface > 1 && n_iface <= kMaxBatch) {
        const Iface &f0 = h->ifs[0];
        bool same = true, turbine = true;
        for (const Iface &f : h->ifs) {
            same = same && f.elem == f0.elem && f.d.physics == f0.d.physics &&
                   f.d.riemann == f0.d.riemann && f.flux_variant == 0 && f.d.N <= kMaxNFast;
            turbine = turbine && (f.NP == 4 || f.NP == 6 || f.NP == 8);
        }
        const bool ns = f0.d.physics == MORTAR_NAVIER_STOKES;
        const int riem = f0.d.riemann == MORTAR_FLUX_ROE;
        h->batched = same;
        h->batch_turbine = turbine && ns && riem && f0.elem == 4;
        if (same)
            h->batch_occ = f0.elem == 8 ? flux_batch_occupancy_f64(ns, riem, h->batch_turbine)
                                        : flux_batch_occupancy_f32(ns, riem, h->batch_turbine);
        // the register-direct batch kernel: FP32, degrees N = 3, 5, 7
        bool rd_ok = same && f0.elem == 4;
        for (const Iface &f : h->ifs) rd_ok = rd_ok && f.lp == 0 && variant_allowed(f, 2);
        h->batch_rd_ok = rd_ok && turbine;
        if (h->batch_rd_ok) h->batch_occ_rd = flux_rd_batch_occupancy_f32(ns, riem);
    }
    *out = h;
    return MORTAR_OK;
}

int mortar_destroy(mortar_handle *h)
{
    if (!h) return MORTAR_ERR_INVALID_ARG;
    (void)hipDeviceSynchronize();
    for (auto &f : h->ifs) free_iface(f);
    delete h;
    return MORTAR_OK;
}

int mortar_update_displacement(mortar_handle *h, const double *disp, void *stream)
{
    if (!h || !disp) return MORTAR_ERR_INVALID_ARG;
    const size_t n_if = h->ifs.size();
    std::vector<int64_t> n(n_if);
    std::vector<double> s(n_if);
    for (size_t i = 0; i < n_if; ++i) {
        const int rc = mortar_decompose_displacement(disp[i], h->ifs[i].d.l_par, &n[i], &s[i]);
        if (rc) return rc;
    }
    return apply_update(h, n.data(), s.data(), (hipStream_t)stream);
}

int mortar_update_displacement_ns(mortar_handle *h, const int64_t *n, const double *s,
                                  void *stream)
{
    if (!h || !n || !s) return MORTAR_ERR_INVALID_ARG;
    for (size_t i = 0; i < h->ifs.size(); ++i)
        if (!(s[i] >= 0.0 && s[i] < 1.0)) return MORTAR_ERR_INVALID_ARG;
    return apply_update(h, n, s, (hipStream_t)stream);
}

int mortar_flux(mortar_handle *h, const void *const *U_s, const void *const *U_m,
                const void *const *G_s, const void *const *G_m, void *const *F_s,
                void *const *F_m, void *stream)
{
    if (!h || !U_s || !U_m || !F_s || !F_m) return MORTAR_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    for (size_t i = 0; i < h->ifs.size(); ++i) {
        const Iface &f = h->ifs[i];
        if (!f.ready) return MORTAR_ERR_NOT_READY;
        const bool ns = f.d.physics == MORTAR_NAVIER_STOKES;
        if (!U_s[i] || !U_m[i] || !F_s[i] || !F_m[i]) return MORTAR_ERR_INVALID_ARG;
        if (ns && (!G_s || !G_m || !G_s[i] || !G_m[i])) return MORTAR_ERR_INVALID_ARG;
    }
    if (h->batched) {
        TRY_HIP(launch_flux_batched(*h, U_s, U_m, G_s, G_m, F_s, F_m, st));
        return MORTAR_OK;
    }
    for (size_t i = 0; i < h->ifs.size(); ++i) {
        const Iface &f = h->ifs[i];
        const bool ns = f.d.physics == MORTAR_NAVIER_STOKES;
        TRY_HIP(launch_flux(f, h->n_cu, U_s[i], U_m[i], ns ? G_s[i] : nullptr,
                            ns ? G_m[i] : nullptr, F_s[i], F_m[i], st));
    }
    return MORTAR_OK;
}

int mortar_lifting(mortar_handle *h, const void *const *U_s, const void *const *U_m,
                   void *const *L_s, void *const *L_m, void *stream)
{
    if (!h || !U_s || !U_m || !L_s || !L_m) return MORTAR_ERR_INVALID_ARG;
    for (size_t i = 0; i < h->ifs.size(); ++i) {
        const Iface &f = h->ifs[i];
        if (!f.ready) return MORTAR_ERR_NOT_READY;
        if (!U_s[i] || !U_m[i] || !L_s[i] || !L_m[i]) return MORTAR_ERR_INVALID_ARG;
        const int64_t nf = std::max<int64_t>(f.d.n_face_static, f.d.n_face_moving);
        if (15 * (int64_t)f.P * nf * (int64_t)f.elem >= ((int64_t)1 << 31)) return MORTAR_ERR_UNSUPPORTED;
    }
    hipStream_t st = (hipStream_t)stream;
    for (size_t i = 0; i < h->ifs.size(); ++i) {
        const Iface &f = h->ifs[i];
        const bool met = f.d_metrics != nullptr, f64 = f.elem == 8;
        if (!f64 && f.d.N <= kMaxNFast) {
            // FP32 up to degree 9: the register-direct body (one wave per 15-face tile;
            // from NP = 8 in the lockstep rounds of the flux launches).  Plane N = 5,
            // 128x64: 18.8 us against 25.6 us for the VALU kernel; annulus N = 7, 512x64:
            // 111.5 us against 145 us (with four free waves instead of the rounds: 165).
            const int tiles_per_row = (f.d.n_par + kRdTileFaces - 1) / kRdTileFaces;
            const int tile_len = (f.d.n_par + tiles_per_row - 1) / tiles_per_row;
            const int n_tiles = tiles_per_row * f.NP * f.d.n_perp;
            const int w = rd_lift_waves(f.NP);
            const int grid = std::max(8, std::min((n_tiles + w - 1) / w, lift_rd_occupancy_f32(f.NP, met) * h->n_cu));
            FluxArgs<float> a;
            int nt = 0;
            fill_args(f, U_s[i], U_m[i], nullptr, nullptr, L_s[i], L_m[i], a, nt);
            a.tiles_per_row = tiles_per_row; a.tile_len = tile_len; a.n_tiles = n_tiles;
            a.cons = nullptr;
            TRY_HIP(launch_lift_rd_f32(a, f.NP, grid, met, st));
            continue;
        }
        // tiles of the lifting kernel's capacity, balanced along the row (fill_args uses
        // the flux launch's tuning, so the fields are set here)
        const int cap = lift_tile_capacity(f.NP, met, f64);
        const int tiles_per_row = (f.d.n_par + cap - 1) / cap;
        const int tile_len = (f.d.n_par + tiles_per_row - 1) / tiles_per_row;
        const int n_tiles = tiles_per_row * f.NP * f.d.n_perp;
        const int grid = std::max(1, std::min(n_tiles, lift_occupancy(f.NP, met, f64) * h->n_cu));
        int nt = 0;
        if (f64) {
            FluxArgs<double> a;
            fill_args(f, U_s[i], U_m[i], nullptr, nullptr, L_s[i], L_m[i], a, nt);
            a.tiles_per_row = tiles_per_row; a.tile_len = tile_len; a.n_tiles = n_tiles;
            TRY_HIP(launch_lift_f64(a, f.NP, grid, met, st));
        } else {
            FluxArgs<float> a;
            fill_args(f, U_s[i], U_m[i], nullptr, nullptr, L_s[i], L_m[i], a, nt);
            a.tiles_per_row = tiles_per_row; a.tile_len = tile_len; a.n_tiles = n_tiles;
            TRY_HIP(launch_lift_f32(a, f.NP, grid, met, st));
        }
    }
    return MORTAR_OK;
}

int mortar_get_displacement(mortar_handle *h, int iface, int64_t *n, double *s)
{
    if (!h || iface < 0 || iface >= (int)h->ifs.size() || !n || !s) return MORTAR_ERR_INVALID_ARG;
    if (!h->ifs[iface].ready) return MORTAR_ERR_NOT_READY;
    *n = h->ifs[iface].n;
    *s = h->ifs[iface].s;
    return MORTAR_OK;
}

int mortar_get_index_map(mortar_handle *h, int iface, int side, int32_t *A, int32_t *m)
{
    if (!h || iface < 0 || iface >= (int)h->ifs.size() || side < 0 || side > 1)
        return MORTAR_ERR_INVALID_ARG;
    const Iface &f = h->ifs[iface];
    if (!f.ready) return MORTAR_ERR_NOT_READY;
    TRY_HIP(hipDeviceSynchronize());
    if (A) TRY_HIP(hipMemcpy(A, f.d_A[side], sizeof(int32_t) * 10 * (size_t)f.F, hipMemcpyDeviceToHost));
    const int nf = side ? f.d.n_face_moving : f.d.n_face_static;
    if (m) TRY_HIP(hipMemcpy(m, f.d_m[side], sizeof(int32_t) * 2 * (size_t)nf, hipMemcpyDeviceToHost));
    return MORTAR_OK;
}

int mortar_get_pairing(mortar_handle *h, int iface, int32_t *pair)
{
    if (!h || iface < 0 || iface >= (int)h->ifs.size() || !pair) return MORTAR_ERR_INVALID_ARG;
    const Iface &f = h->ifs[iface];
    if (!f.ready) return MORTAR_ERR_NOT_READY;
    TRY_HIP(hipDeviceSynchronize());
    TRY_HIP(launch_pairing(f, nullptr));
    TRY_HIP(hipDeviceSynchronize());
    TRY_HIP(hipMemcpy(pair, f.d_pair, sizeof(int32_t) * 2 * (size_t)f.d.n_par, hipMemcpyDeviceToHost));
    return MORTAR_OK;
}

int mortar_get_projection(mortar_handle *h, int iface, double *Pf, double *Pb)
{
    if (!h || iface < 0 || iface >= (int)h->ifs.size()) return MORTAR_ERR_INVALID_ARG;
    const Iface &f = h->ifs[iface];
    if (!f.ready) return MORTAR_ERR_NOT_READY;
    TRY_HIP(launch_assemble(f, nullptr));
    TRY_HIP(hipDeviceSynchronize());
    const size_t nn = (size_t)4 * f.NP * f.NP;
    if (Pf) TRY_HIP(hipMemcpy(Pf, f.d_params + off_f64(f.NP), sizeof(double) * nn, hipMemcpyDeviceToHost));
    if (Pb)
        TRY_HIP(hipMemcpy(Pb, f.d_params + off_f64(f.NP) + sizeof(double) * nn, sizeof(double) * nn,
                          hipMemcpyDeviceToHost));
    return MORTAR_OK;
}

int mortar_conservation_device(mortar_handle *h, const void *const *F_s, const void *const *F_m,
                               double *d_out, void *stream)
{
    if (!h || !F_s || !F_m || !d_out) return MORTAR_ERR_INVALID_ARG;
    for (size_t i = 0; i < h->ifs.size(); ++i)
        if (!F_s[i] || !F_m[i]) return MORTAR_ERR_INVALID_ARG;
    // every interface's partials written by its last flux launch into these outputs: one
    // final launch for all of them
    const size_t n_if = h->ifs.size();
    bool all_fused = n_if > 1 && n_if <= (size_t)kMaxConsBatch;
    for (size_t i = 0; i < n_if && all_fused; ++i) {
        const Iface &f = h->ifs[i];
        all_fused = f.cons_nb > 0 && f.cons_Fs == F_s[i] && f.cons_Fm == F_m[i];
    }
    if (all_fused) {
        const Iface *fs[kMaxConsBatch];
        double *outs[kMaxConsBatch];
        for (size_t i = 0; i < n_if; ++i) {
            fs[i] = &h->ifs[i];
            outs[i] = d_out + 15 * i;
        }
        TRY_HIP(launch_conservation_final_batch(fs, outs, (int)n_if, (hipStream_t)stream));
        return MORTAR_OK;
    }
    for (size_t i = 0; i < n_if; ++i)
        TRY_HIP(launch_conservation_any(h->ifs[i], F_s[i], F_m[i], d_out + 15 * i, (hipStream_t)stream));
    return MORTAR_OK;
}

int mortar_conservation_device_noalloc(mortar_handle *h, const void *const *F_s,
                                       const void *const *F_m, double *d_out, void *stream)
{
    if (!h || !F_s || !F_m || !d_out) return MORTAR_ERR_INVALID_ARG;
    if (h->ifs.size() > (size_t)kStaticConsIfaces) return MORTAR_ERR_UNSUPPORTED;
    if (!h->static_scratch) return MORTAR_ERR_HIP;
    for (size_t i = 0; i < h->ifs.size(); ++i)
        if (!F_s[i] || !F_m[i]) return MORTAR_ERR_INVALID_ARG;
    for (size_t i = 0; i < h->ifs.size(); ++i)
        TRY_HIP(launch_conservation_static(h->ifs[i], (int)i, h->static_scratch, F_s[i], F_m[i],
                                           d_out + 15 * i, (hipStream_t)stream));
    return MORTAR_OK;
}

int mortar_conservation(mortar_handle *h, const void *const *F_s, const void *const *F_m,
                        double *out, void *stream)
{
    if (!h || !F_s || !F_m || !out) return MORTAR_ERR_INVALID_ARG;
    hipStream_t st = (hipStream_t)stream;
    for (size_t i = 0; i < h->ifs.size(); ++i) {
        if (!F_s[i] || !F_m[i]) return MORTAR_ERR_INVALID_ARG;
        const Iface &f = h->ifs[i];
        TRY_HIP(launch_conservation_any(f, F_s[i], F_m[i], f.d_cons_out, st));
        TRY_HIP(hipMemcpyAsync(out + 15 * i, f.d_cons_out, sizeof(double) * 15,
                               hipMemcpyDeviceToHost, st));
    }
    TRY_HIP(hipStreamSynchronize(st));
    return MORTAR_OK;
}

// The capture behind mortar_graph_create and mortar_graph_create_cons (d_cons non-null:
// the stage's conservation sums into d_cons after the flux launches).
static int graph_create(mortar_handle *h, const void *const *U_s, const void *const *U_m,
                        const void *const *G_s, const void *const *G_m, void *const *F_s,
                        void *const *F_m, double *d_cons, mortar_graph **out)
{
    if (!h || !out || !U_s || !U_m || !F_s || !F_m) return MORTAR_ERR_INVALID_ARG;
    const size_t n_if = h->ifs.size();
    mortar_graph *g = new (std::nothrow) mortar_graph();
    if (!g) return MORTAR_ERR_OOM;
    g->h = h;
    g->epoch = h->tune_epoch;
    for (size_t i = 0; i < n_if; ++i) {
        g->Us.push_back(U_s[i]);
        g->Um.push_back(U_m[i]);
        g->Gs.push_back(G_s ? G_s[i] : nullptr);
        g->Gm.push_back(G_m ? G_m[i] : nullptr);
        g->Fs.push_back(F_s[i]);
        g->Fm.push_back(F_m[i]);
    }
    hipStream_t cs = nullptr;
    int rc = MORTAR_OK;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) rc = MORTAR_ERR_HIP;
    if (rc == MORTAR_OK && hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess)
        rc = MORTAR_ERR_HIP;
    if (rc == MORTAR_OK) {
        int frc = mortar_flux(h, g->Us.data(), g->Um.data(), g->Gs.data(), g->Gm.data(),
                              g->Fs.data(), g->Fm.data(), cs);
        if (frc == MORTAR_OK && d_cons)
            frc = mortar_conservation_device(h, g->Fs.data(), g->Fm.data(), d_cons, cs);
        hipGraph_t graph = nullptr;
        const hipError_t e = hipStreamEndCapture(cs, &graph);
        g->graph = graph;
        if (frc != MORTAR_OK) rc = frc;
        else if (e != hipSuccess || !graph) rc = MORTAR_ERR_HIP;
    }
    if (rc == MORTAR_OK) {
        size_t nn = 0;
        if (hipGraphGetNodes(g->graph, nullptr, &nn) != hipSuccess) rc = MORTAR_ERR_HIP;
        std::vector<hipGraphNode_t> all(nn);
        if (rc == MORTAR_OK && nn && hipGraphGetNodes(g->graph, all.data(), &nn) != hipSuccess)
            rc = MORTAR_ERR_HIP;
        // the flux nodes (updated per replay) and the conservation nodes (fixed); no
        // memset node may be part of a replayed graph
        size_t n_cons = 0;
        for (size_t i = 0; rc == MORTAR_OK && i < nn; ++i) {
            hipGraphNodeType t;
            if (hipGraphNodeGetType(all[i], &t) != hipSuccess) {
                rc = MORTAR_ERR_HIP;
            } else if (t == hipGraphNodeTypeMemset) {
                rc = MORTAR_ERR_UNSUPPORTED;
            } else if (t == hipGraphNodeTypeKernel) {
                hipKernelNodeParams p{};
                if (hipGraphKernelNodeGetParams(all[i], &p) != hipSuccess) rc = MORTAR_ERR_HIP;
                else if (is_conservation_kernel(p.func)) ++n_cons;
                else g->nodes.push_back(all[i]);
            }
        }
        const size_t want = h->batched ? 1 : n_if;
        if (rc == MORTAR_OK && g->nodes.size() != want) rc = MORTAR_ERR_UNSUPPORTED;
        if (rc == MORTAR_OK && (d_cons ? n_cons == 0 : n_cons != 0)) rc = MORTAR_ERR_UNSUPPORTED;
    }
    if (rc == MORTAR_OK && hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess)
        rc = MORTAR_ERR_HIP;
    if (cs) (void)hipStreamDestroy(cs);
    // the captured launch has not run: no partials of it exist until a replay writes them
    // (mortar_graph_launch records them per replay)
    for (auto &f : h->ifs) f.cons_nb = 0;
    if (rc != MORTAR_OK) {
        mortar_graph_destroy(g);
        return rc;
    }
    *out = g;
    return MORTAR_OK;
}

int mortar_graph_create(mortar_handle *h, const void *const *U_s, const void *const *U_m,
                        const void *const *G_s, const void *const *G_m, void *const *F_s,
                        void *const *F_m, mortar_graph **out)
{
    return graph_create(h, U_s, U_m, G_s, G_m, F_s, F_m, nullptr, out);
}

int mortar_graph_create_cons(mortar_handle *h, const void *const *U_s, const void *const *U_m,
                             const void *const *G_s, const void *const *G_m, void *const *F_s,
                             void *const *F_m, double *d_cons, mortar_graph **out)
{
    if (!d_cons) return MORTAR_ERR_INVALID_ARG;
    return graph_create(h, U_s, U_m, G_s, G_m, F_s, F_m, d_cons, out);
}

}  // extern "C"

template <typename Args>
static int set_node_args(mortar_graph *g, size_t node, Args &args)
{
    hipKernelNodeParams p;
    if (hipGraphKernelNodeGetParams(g->nodes[node], &p) != hipSuccess) return MORTAR_ERR_HIP;
    void *kp[1] = {&args};
    p.kernelParams = kp;
    p.extra = nullptr;
    if (hipGraphExecKernelNodeSetParams(g->exec, g->nodes[node], &p) != hipSuccess)
        return MORTAR_ERR_HIP;
    return MORTAR_OK;
}

extern "C" {

int mortar_graph_launch(mortar_graph *g, const double *disp, void *stream)
{
    if (!g || !g->exec || !disp) return MORTAR_ERR_INVALID_ARG;
    mortar_handle *h = g->h;
    if (g->epoch != h->tune_epoch) return MORTAR_ERR_UNSUPPORTED;   // captured before a retune
    int rc = mortar_update_displacement(h, disp, stream);
    if (rc) return rc;
    const size_t n_if = h->ifs.size();
    if (h->batched) {
        const bool f64 = h->ifs[0].elem == 8;
        auto build = [&](auto &b) {
            b.n_if = (int)n_if;
            int total = 0;
            for (size_t i = 0; i < n_if; ++i) {
                int nt = 0;
                fill_args(h->ifs[i], g->Us[i], g->Um[i], g->Gs[i], g->Gm[i], g->Fs[i], g->Fm[i],
                          b.a[i], nt);
                h->ifs[i].cons_nb = 0;
                b.np[i] = h->ifs[i].NP;
                b.met[i] = h->ifs[i].d_metrics != nullptr;
                total += nt;
            }
            // the register-direct batch kernel writes each interface's partials (the grid
            // is the one the captured launch was given)
            if (h->batch_variant == 2) {
                const int grid = rd_batch_grid(*h, total);
                for (size_t i = 0; i < n_if; ++i) set_cons(h->ifs[i], b.a[i], grid, g->Fs[i], g->Fm[i]);
            }
        };
        if (f64) {
            BatchArgs<double> b;
            build(b);
            rc = set_node_args(g, 0, b);
        } else {
            BatchArgs<float> b;
            build(b);
            rc = set_node_args(g, 0, b);
        }
    } else {
        for (size_t i = 0; i < n_if && rc == MORTAR_OK; ++i) {
            int nt = 0;
            if (h->ifs[i].elem == 8) {
                FluxArgs<double> a;
                fill_args(h->ifs[i], g->Us[i], g->Um[i], g->Gs[i], g->Gm[i], g->Fs[i], g->Fm[i], a, nt);
                h->ifs[i].cons_nb = 0;
                const int grid = h->ifs[i].flux_variant == 2 ? rd_grid_of(h->ifs[i], h->n_cu, nt)
                                                             : tiled_grid(h->ifs[i], h->n_cu, nt);
                set_cons(h->ifs[i], a, grid, g->Fs[i], g->Fm[i]);
                rc = set_node_args(g, i, a);
            } else {
                FluxArgs<float> a;
                fill_args(h->ifs[i], g->Us[i], g->Um[i], g->Gs[i], g->Gm[i], g->Fs[i], g->Fm[i], a, nt);
                h->ifs[i].cons_nb = 0;
                const int grid = h->ifs[i].flux_variant == 2 ? rd_grid_of(h->ifs[i], h->n_cu, nt)
                                                             : tiled_grid(h->ifs[i], h->n_cu, nt);
                set_cons(h->ifs[i], a, grid, g->Fs[i], g->Fm[i]);
                rc = set_node_args(g, i, a);
            }
        }
    }
    if (rc) return rc;
    TRY_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream));
    return MORTAR_OK;
}

// ---- autotuner ------------------------------------------------------------------------

}  // extern "C"

// Average time of one launch (ms): one warm-up, then reps launches between two events.
// Device buffer larger than the caches (4 MB L2 per XCD, the 256 MB Infinity Cache),
// filled before every timed call so that each starts with its inputs in HBM, as a stage
// with fresh data does; released when the autotuner returns.
struct CacheFlush {
    static constexpr size_t kBytes = (size_t)512 << 20;
    void *buf = nullptr;
    CacheFlush()
    {
        if (hipMalloc(&buf, kBytes) != hipSuccess) buf = nullptr;   // then timed warm
    }
    ~CacheFlush()
    {
        if (buf) (void)hipFree(buf);
    }
    hipError_t run(int r, hipStream_t st) const
    {
        return buf ? hipMemsetAsync(buf, r & 0xff, kBytes, st) : hipSuccess;
    }
};

// Average time of one call of launch() over reps timed calls (each between its own pair
// of events, after a cache flush), following one untimed call.
template <typename F>
static hipError_t time_launches(F &&launch, int reps, hipStream_t st, float &ms, const CacheFlush &cf)
{
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t err = hipEventCreate(&e0);
    if (err == hipSuccess) err = hipEventCreate(&e1);
    if (err == hipSuccess) err = launch();
    float total = 0.f;
    for (int r = 0; r < reps && err == hipSuccess; ++r) {
        err = cf.run(r, st);
        if (err == hipSuccess) err = hipEventRecord(e0, st);
        if (err == hipSuccess) err = launch();
        if (err == hipSuccess) err = hipEventRecord(e1, st);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        float t = 0.f;
        if (err == hipSuccess) err = hipEventElapsedTime(&t, e0, e1);
        total += t;
    }
    ms = total / (float)reps;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return err;
}

// Three tile lengths per capacity: the largest, about two thirds and about half.
static std::vector<int> tile_candidates(int cap)
{
    std::vector<int> t = {cap, std::max(2, (2 * cap + 2) / 3), std::max(2, (cap + 1) / 2)};
    std::sort(t.begin(), t.end());
    t.erase(std::unique(t.begin(), t.end()), t.end());
    return t;
}

static int vmax_tile(const Iface &f, int variant)
{
    const bool ns = f.d.physics == MORTAR_NAVIER_STOKES, met = f.d_metrics != nullptr;
    if (variant == 3) return flux_wide_tile_capacity_f32(f.NP, ns, met);
    if (variant == 4) return flux_hyb_tile_capacity_f32(f.NP, ns, met);
    if (variant != 0) return 15;
    return f.elem == 8 ? flux_tile_capacity_f64(f.NP, ns, met) : flux_tile_capacity_f32(f.NP, ns, met);
}

static int autotune_run(mortar_handle *h, const void *const *U_s, const void *const *U_m,
                        const void *const *G_s, const void *const *G_m, void *const *F_s,
                        void *const *F_m, int reps, hipStream_t st);

extern "C" {

int mortar_autotune(mortar_handle *h, const void *const *U_s, const void *const *U_m,
                    const void *const *G_s, const void *const *G_m, void *const *F_s,
                    void *const *F_m, int reps, void *stream)
{
    if (!h || !U_s || !U_m || !F_s || !F_m) return MORTAR_ERR_INVALID_ARG;
    if (reps <= 0) reps = 5;
    hipStream_t st = (hipStream_t)stream;
    const size_t n_if = h->ifs.size();
    for (size_t i = 0; i < n_if; ++i) {
        const Iface &f = h->ifs[i];
        if (!f.ready) return MORTAR_ERR_NOT_READY;
        const bool ns = f.d.physics == MORTAR_NAVIER_STOKES;
        if (!U_s[i] || !U_m[i] || !F_s[i] || !F_m[i]) return MORTAR_ERR_INVALID_ARG;
        if (ns && (!G_s || !G_m || !G_s[i] || !G_m[i])) return MORTAR_ERR_INVALID_ARG;
    }
    const int rc = autotune_run(h, U_s, U_m, G_s, G_m, F_s, F_m, reps, st);
    return rc;
}

}  // extern "C"

// The tuning state of a handle, saved before the autotuner times its candidates and put
// back when a HIP error ends it early (the handle then launches as before the call).
struct TuningState {
    int batch_variant, tune_grid_batch;
    unsigned epoch;
    std::vector<int> variant, occ, tile, grid;
    explicit TuningState(const Handle &h)
        : batch_variant(h.batch_variant), tune_grid_batch(h.tune_grid_batch), epoch(h.tune_epoch)
    {
        for (const Iface &f : h.ifs) {
            variant.push_back(f.flux_variant);
            occ.push_back(f.flux_occ);
            tile.push_back(f.tune_tile);
            grid.push_back(f.tune_grid);
        }
    }
    void restore(Handle &h) const
    {
        h.batch_variant = batch_variant;
        h.tune_grid_batch = tune_grid_batch;
        h.tune_epoch = epoch;
        for (size_t i = 0; i < h.ifs.size(); ++i) {
            h.ifs[i].flux_variant = variant[i];
            h.ifs[i].flux_occ = occ[i];
            h.ifs[i].tune_tile = tile[i];
            h.ifs[i].tune_grid = grid[i];
            h.ifs[i].cons_nb = 0;
        }
    }
};

static int autotune_timed(mortar_handle *h, const void *const *U_s, const void *const *U_m,
                          const void *const *G_s, const void *const *G_m, void *const *F_s,
                          void *const *F_m, int reps, hipStream_t st);

static int autotune_run(mortar_handle *h, const void *const *U_s, const void *const *U_m,
                        const void *const *G_s, const void *const *G_m, void *const *F_s,
                        void *const *F_m, int reps, hipStream_t st)
{
    const TuningState saved(*h);
    const int rc = autotune_timed(h, U_s, U_m, G_s, G_m, F_s, F_m, reps, st);
    if (rc != MORTAR_OK) saved.restore(*h);
    return rc;
}

static int autotune_timed(mortar_handle *h, const void *const *U_s, const void *const *U_m,
                          const void *const *G_s, const void *const *G_m, void *const *F_s,
                          void *const *F_m, int reps, hipStream_t st)
{
    const size_t n_if = h->ifs.size();
    h->tune_epoch++;
    const CacheFlush flush;
    float ms = 0.f;
    // MORTAR_TUNE_LOG=1 prints every candidate's time to stderr
    const bool log = std::getenv("MORTAR_TUNE_LOG") != nullptr;
    auto note = [&](int iface, int v, int t, int g) {
        if (log) std::fprintf(stderr, "[autotune] iface %d variant %d tile %d grid %d: %.2f us\n", iface, v, t, g, 1e3 * ms);
    };
    if (h->batched) {
        // a candidate's time includes the stage's conservation sums (the partials some
        // batch kernels write with the fluxes, else a pass over the arrays)
        auto run = [&]() {
            hipError_t e = launch_flux_batched(*h, U_s, U_m, G_s, G_m, F_s, F_m, st);
            for (size_t i = 0; i < n_if && e == hipSuccess; ++i)
                e = launch_conservation_any(h->ifs[i], F_s[i], F_m[i], h->ifs[i].d_cons_out, st);
            return e;
        };
        auto set_variant = [&](int v) {
            h->batch_variant = v;
            for (Iface &f : h->ifs) {
                f.flux_variant = v;
                f.flux_occ = variant_occupancy(f, v);
            }
        };
        // per batch kernel: coordinate descent over each interface's tile length, then
        // the grid; keep the best batch kernel with its settings
        float best_all = 1e30f;
        int best_v = 0, best_grid = 0;
        std::vector<int> best_tiles(n_if, 0);
        for (int v : {0, 2}) {
            if (v == 2 && !h->batch_rd_ok) continue;
            set_variant(v);
            h->tune_grid_batch = 0;
            for (Iface &f : h->ifs) f.tune_tile = 0;
            float best = 1e30f;
            for (size_t i = 0; i < n_if; ++i) {
                Iface &f = h->ifs[i];
                int best_t = 0;
                float bi = 1e30f;
                for (int t : tile_candidates(vmax_tile(f, v))) {
                    f.tune_tile = t;
                    TRY_HIP(time_launches(run, reps, st, ms, flush));
                    note((int)i, v, t, h->tune_grid_batch);
                    if (ms < bi) { bi = ms; best_t = t; }
                }
                f.tune_tile = best_t;
            }
            const int occ = v == 2 ? h->batch_occ_rd : h->batch_occ;
            int best_g = 0;
            float bg = 1e30f;
            for (int k = occ; k >= 1; --k) {
                h->tune_grid_batch = k == occ ? 0 : k * h->n_cu;
                TRY_HIP(time_launches(run, reps, st, ms, flush));
                note(-1, v, 0, h->tune_grid_batch);
                if (ms < bg) { bg = ms; best_g = h->tune_grid_batch; }
            }
            best = bg;
            if (best < best_all) {
                best_all = best;
                best_v = v;
                best_grid = best_g;
                for (size_t i = 0; i < n_if; ++i) best_tiles[i] = h->ifs[i].tune_tile;
            }
        }
        set_variant(best_v);
        h->tune_grid_batch = best_grid;
        for (size_t i = 0; i < n_if; ++i) h->ifs[i].tune_tile = best_tiles[i];
        return MORTAR_OK;
    }
    for (size_t i = 0; i < n_if; ++i) {
        Iface &f = h->ifs[i];
        const bool ns = f.d.physics == MORTAR_NAVIER_STOKES;
        // a candidate's time includes the stage's conservation sums: fused into the VALU
        // kernels' launch, a separate pass after the others
        auto run = [&]() {
            hipError_t e = launch_flux(f, h->n_cu, U_s[i], U_m[i], ns ? G_s[i] : nullptr,
                                       ns ? G_m[i] : nullptr, F_s[i], F_m[i], st);
            if (e == hipSuccess) e = launch_conservation_any(f, F_s[i], F_m[i], f.d_cons_out, st);
            return e;
        };
        int best_v = f.flux_variant, best_t = f.tune_tile;
        float best = 1e30f;
        for (int v = 0; v <= 4; ++v) {
            if (!variant_allowed(f, v)) continue;
            f.flux_variant = v;
            f.flux_occ = variant_occupancy(f, v);
            f.tune_grid = 0;
            for (int t : tile_candidates(vmax_tile(f, v))) {
                f.tune_tile = t;
                TRY_HIP(time_launches(run, reps, st, ms, flush));
                note((int)i, v, t, 0);
                if (ms < best) { best = ms; best_v = v; best_t = t; }
            }
        }
        f.flux_variant = best_v;
        f.flux_occ = variant_occupancy(f, best_v);
        f.tune_tile = best_t;
    }
    return MORTAR_OK;
}

extern "C" {

int mortar_get_tuning(const mortar_handle *h, int iface, mortar_tuning *out)
{
    if (!h || !out || iface < 0 || iface >= (int)h->ifs.size()) return MORTAR_ERR_INVALID_ARG;
    const Iface &f = h->ifs[iface];
    out->variant = h->batched ? h->batch_variant : f.flux_variant;
    out->tile_len = f.tune_tile;
    out->grid = h->batched ? h->tune_grid_batch : f.tune_grid;
    out->reserved = 0;
    return MORTAR_OK;
}

int mortar_set_tuning(mortar_handle *h, int iface, const mortar_tuning *t)
{
    if (!h || !t || iface < 0 || iface >= (int)h->ifs.size()) return MORTAR_ERR_INVALID_ARG;
    if (t->tile_len < 0 || t->grid < 0 || (t->grid > 0 && t->grid < 8)) return MORTAR_ERR_INVALID_ARG;
    Iface &f = h->ifs[iface];
    if (!variant_allowed(f, t->variant)) return MORTAR_ERR_INVALID_ARG;
    if (h->batched && !(t->variant == 0 || (t->variant == 2 && h->batch_rd_ok)))
        return MORTAR_ERR_INVALID_ARG;
    h->tune_epoch++;
    if (h->batched) {
        // the kernel variant and the grid belong to the whole batch
        h->batch_variant = t->variant;
        for (Iface &g : h->ifs) {
            g.flux_variant = t->variant;
            g.flux_occ = variant_occupancy(g, t->variant);
        }
        h->tune_grid_batch = t->grid;
    } else {
        f.flux_variant = t->variant;
        f.flux_occ = variant_occupancy(f, t->variant);
        f.tune_grid = t->grid;
    }
    f.tune_tile = t->tile_len;
    return MORTAR_OK;
}

int mortar_graph_destroy(mortar_graph *g)
{
    if (!g) return MORTAR_ERR_INVALID_ARG;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
    return MORTAR_OK;
}

}  // extern "C"

namespace mortar {

// Kernel arguments of one interface for the VALU or matrix-core kernel.
template <typename T>
void fill_args(const Iface &f, const void *Us, const void *Um, const void *Gs,
                      const void *Gm, void *Fs, void *Fm, FluxArgs<T> &a, int &n_tiles)
{
    const bool ns = f.d.physics == MORTAR_NAVIER_STOKES;
    const bool met = f.d_metrics != nullptr;
    const double gm1 = f.d.gamma - 1.0;
    const double kfac = ns ? f.d.mu * f.d.gamma / (gm1 * f.d.Pr) : 0.0;
    const int64_t np = f.d.n_par;
    int cap = f.flux_variant == 3 ? flux_wide_tile_capacity_f32(f.NP, ns, met)
            : f.flux_variant == 4 ? flux_hyb_tile_capacity_f32(f.NP, ns, met)
            : f.flux_variant != 0 ? kRdTileFaces
            : (f.elem == 8 ? flux_tile_capacity_f64(f.NP, ns, met)
                           : flux_tile_capacity_f32(f.NP, ns, met));
    if (f.tune_tile > 0) cap = std::min(cap, f.tune_tile);
    // balanced tiles: as few as the capacity allows, all of nearly equal length
    const int tiles_per_row = (f.d.n_par + cap - 1) / cap;
    const int tile_len = (f.d.n_par + tiles_per_row - 1) / tiles_per_row;
    n_tiles = tiles_per_row * f.NP * f.d.n_perp;
    a.Us = (const T *)Us; a.Um = (const T *)Um;
    a.Gs = (const T *)Gs; a.Gm = (const T *)Gm;
    a.met = (const T *)f.d_metrics;
    a.Fs = (T *)Fs; a.Fm = (T *)Fm;
    a.fid_s = f.d_fid_s; a.fid_m = f.d_fid_m;
    a.basis = f.d_basis;
    a.s = f.s;
    a.nmod = (int)(((f.n % np) + np) % np);
    a.n_par = f.d.n_par; a.n_perp = f.d.n_perp;
    a.nfs = f.d.n_face_static; a.nfm = f.d.n_face_moving;
    a.tiles_per_row = tiles_per_row;
    a.tile_len = tile_len;
    a.n_tiles = n_tiles;
    a.nx = (T)f.d.normal[0]; a.ny = (T)f.d.normal[1]; a.nz = (T)f.d.normal[2];
    a.dS = (T)f.d.dS;
    a.gas = {(T)gm1, (T)f.d.gamma, (T)(ns ? f.d.mu : 0.0), (T)kfac};
    a.cons = nullptr;
}

// Grid of the register-direct kernel: one tile per wave, rd_waves() waves per workgroup,
// at most the resident workgroups, at least one workgroup per XCD.
static int rd_grid_of(const Iface &f, int n_cu, int nt)
{
    if (f.tune_grid > 0) return std::max(8, f.tune_grid);
    const int w = rd_waves((int)f.elem, f.d.physics == MORTAR_NAVIER_STOKES, f.NP);
    return std::max(8, std::min((nt + w - 1) / w, f.flux_occ * n_cu));
}

// Persistent grid of the LDS-tiled kernels: at least min(8, n_tiles) workgroups so that
// every XCD's share of the tiles has workers (TileCursor).
static int tiled_grid(const Iface &f, int n_cu, int nt)
{
    if (f.tune_grid > 0) return std::max(std::min(8, nt), std::min(nt, f.tune_grid));
    return std::max(1, std::min(nt, f.flux_occ * n_cu));
}

// Kernels that also write the conservation partials of their launch: the VALU-projection
// kernels (variants 0 and 3), and the register-direct kernels with 4-byte data (FP32,
// bf16, fp16); record which outputs the partials belong to.
static bool writes_partials(const Iface &f, int variant)
{
    return variant == 0 || variant == 3 || (variant == 2 && f.elem == 4);
}

template <typename T>
static void set_cons(const Iface &f, FluxArgs<T> &a, int grid, const void *Fs, const void *Fm)
{
    const bool fused = writes_partials(f, f.flux_variant) && grid <= kConsGridMax;
    a.cons = fused ? f.d_cons_wg : nullptr;
    f.cons_Fs = fused ? Fs : nullptr;
    f.cons_Fm = fused ? Fm : nullptr;
    f.cons_nb = fused ? grid : 0;
}

hipError_t launch_flux(const Iface &f, int n_cu, const void *Us, const void *Um, const void *Gs,
                       const void *Gm, void *Fs, void *Fm, hipStream_t st)
{
    const bool ns = f.d.physics == MORTAR_NAVIER_STOKES;
    const bool met = f.d_metrics != nullptr;
    const int riem = f.d.riemann == MORTAR_FLUX_ROE ? 1 : 0;
    int n_tiles = 0;
    f.cons_nb = 0;
    if (f.flux_variant == 2) {
        // one tile per wave, rd_waves() waves per workgroup; at least one workgroup per XCD
        auto rd_grid = [&](int nt) { return rd_grid_of(f, n_cu, nt); };
        if (f.elem == 8) {
            FluxArgs<double> a;
            fill_args(f, Us, Um, Gs, Gm, Fs, Fm, a, n_tiles);
            const int grid = rd_grid(n_tiles);
            set_cons(f, a, grid, Fs, Fm);
            return launch_flux_rd_f64(a, f.NP, grid, ns, met, riem, st);
        }
        FluxArgs<float> a;
        fill_args(f, Us, Um, Gs, Gm, Fs, Fm, a, n_tiles);
        const int grid = rd_grid(n_tiles);
        set_cons(f, a, grid, Fs, Fm);
        if (f.lp == 1) return launch_flux_rd_bf16(a, f.NP, grid, ns, met, riem, st);
        if (f.lp == 2) return launch_flux_rd_fp16(a, f.NP, grid, ns, met, riem, st);
        return launch_flux_rd_f32(a, f.NP, grid, ns, met, riem, st);
    }
    if (f.elem == 8) {
        FluxArgs<double> a;
        fill_args(f, Us, Um, Gs, Gm, Fs, Fm, a, n_tiles);
        const int grid = tiled_grid(f, n_cu, n_tiles);
        set_cons(f, a, grid, Fs, Fm);
        return f.flux_variant == 1 ? launch_flux_mfma_f64(a, f.NP, grid, ns, met, riem, st)
                                   : launch_flux_f64(a, f.NP, grid, ns, met, riem, st);
    }
    FluxArgs<float> a;
    fill_args(f, Us, Um, Gs, Gm, Fs, Fm, a, n_tiles);
    const int grid = tiled_grid(f, n_cu, n_tiles);
    set_cons(f, a, grid, Fs, Fm);
    if (f.flux_variant == 3) return launch_flux_wide_f32(a, f.NP, grid, ns, met, riem, st);
    if (f.flux_variant == 4) return launch_flux_hyb_f32(a, f.NP, grid, ns, met, riem, st);
    return f.flux_variant == 1 ? launch_flux_mfma_f32(a, f.NP, grid, ns, met, riem, st)
                               : launch_flux_f32(a, f.NP, grid, ns, met, riem, st);
}

// Grid of the register-direct batch kernel for total tiles.
static int rd_batch_grid(const Handle &h, int total)
{
    if (h.tune_grid_batch > 0) return std::max(8, h.tune_grid_batch);
    return std::max(8, std::min((total + kRdBatchWaves - 1) / kRdBatchWaves, h.batch_occ_rd * h.n_cu));
}

hipError_t launch_flux_batched(const Handle &h, const void *const *Us, const void *const *Um,
                               const void *const *Gs, const void *const *Gm, void *const *Fs,
                               void *const *Fm, hipStream_t st)
{
    const Iface &f0 = h.ifs[0];
    const bool ns = f0.d.physics == MORTAR_NAVIER_STOKES;
    const int riem = f0.d.riemann == MORTAR_FLUX_ROE ? 1 : 0;
    int total = 0;
    auto build = [&](auto &b) {
        b.n_if = (int)h.ifs.size();
        for (int i = 0; i < b.n_if; ++i) {
            const Iface &f = h.ifs[i];
            int nt = 0;
            fill_args(f, Us[i], Um[i], ns ? Gs[i] : nullptr, ns ? Gm[i] : nullptr, Fs[i], Fm[i],
                      b.a[i], nt);
            f.cons_nb = 0;                       // the batched kernels write no partials
            b.np[i] = f.NP;
            b.met[i] = f.d_metrics != nullptr;
            total += nt;
        }
    };
    auto grid_of = [&](int nt) {
        if (h.tune_grid_batch > 0) return std::max(std::min(8, nt), std::min(nt, h.tune_grid_batch));
        return std::max(1, std::min(nt, h.batch_occ * h.n_cu));
    };
    if (h.batch_variant == 2) {
        // one tile per wave, rd_waves() waves per workgroup; at least one workgroup per XCD
        BatchArgs<float> b;
        build(b);
        const int grid = rd_batch_grid(h, total);
        for (int i = 0; i < b.n_if; ++i) set_cons(h.ifs[i], b.a[i], grid, Fs[i], Fm[i]);
        return launch_flux_rd_batch_f32(b, grid, ns, riem, st);
    }
    if (f0.elem == 8) {
        BatchArgs<double> b;
        build(b);
        const int grid = grid_of(total);
        return launch_flux_batch_f64(b, grid, ns, riem, h.batch_turbine, st);
    }
    BatchArgs<float> b;
    build(b);
    const int grid = grid_of(total);
    return launch_flux_batch_f32(b, grid, ns, riem, h.batch_turbine, st);
}

}  // namespace mortar
