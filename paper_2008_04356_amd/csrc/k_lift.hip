// Instantiations of the BR1 lifting surface kernel (VALU projections), FP32 and FP64,
// with the LDS budget of the VALU flux kernel of the same element type.  Compiled twice:
// N = 1..9 here, N = 10..15 with MORTAR_LIFT_HIGH_DEGREES defined (k_lift_hi.hip).
#include "k_flux.h"

namespace mortar {

namespace {

template <typename T, int NP, bool MET>
hipError_t lift_go(const FluxArgs<T> &a, int grid, hipStream_t st)
{
    hipLaunchKernelGGL((k_mortar_lift<T, NP, MET, lds_budget<T>()>), dim3(grid), dim3(kFluxThreads), 0, st, a);
    return hipGetLastError();
}

template <typename T, int NP, bool MET>
int lift_occ1()
{
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, reinterpret_cast<const void *>(&k_mortar_lift<T, NP, MET, lds_budget<T>()>), kFluxThreads, 0) !=
        hipSuccess)
        return 1;
    return nb > 0 ? nb : 1;
}

template <typename T, int NP>
int lift_cap(bool met)
{
    return met ? FluxCfg<T, NP, false, true, lds_budget<T>(), true>::TF
               : FluxCfg<T, NP, false, false, lds_budget<T>(), true>::TF;
}

template <typename T, int LO, int HI>
struct LiftLaunch {
    static int occupancy(int NP, bool met)
    {
        return np_dispatch<LO, HI, int>(NP, 1, [&](auto c) {
            constexpr int np = decltype(c)::value;
            return met ? lift_occ1<T, np, true>() : lift_occ1<T, np, false>();
        });
    }
    static int capacity(int NP, bool met)
    {
        return np_dispatch<LO, HI, int>(NP, 0, [&](auto c) { return lift_cap<T, decltype(c)::value>(met); });
    }
    static hipError_t launch(const FluxArgs<T> &a, int NP, int grid, bool met, hipStream_t st)
    {
        return np_dispatch<LO, HI, hipError_t>(NP, hipErrorInvalidValue, [&](auto c) {
            constexpr int np = decltype(c)::value;
            return met ? lift_go<T, np, true>(a, grid, st) : lift_go<T, np, false>(a, grid, st);
        });
    }
};

}  // namespace

#ifdef MORTAR_LIFT_HIGH_DEGREES
// N = 10..15
using L32 = LiftLaunch<float, kMaxNFast + 2, kMaxNP>;
using L64 = LiftLaunch<double, kMaxNFast + 2, kMaxNP>;

int lift_occupancy_hi(int NP, bool met, bool f64)
{
    return f64 ? L64::occupancy(NP, met) : L32::occupancy(NP, met);
}

int lift_tile_capacity_hi(int NP, bool met, bool f64)
{
    return f64 ? L64::capacity(NP, met) : L32::capacity(NP, met);
}

hipError_t launch_lift_hi_f32(const FluxArgs<float> &a, int NP, int grid, bool met, hipStream_t st)
{
    return L32::launch(a, NP, grid, met, st);
}

hipError_t launch_lift_hi_f64(const FluxArgs<double> &a, int NP, int grid, bool met, hipStream_t st)
{
    return L64::launch(a, NP, grid, met, st);
}
#else
using L32 = LiftLaunch<float, 2, kMaxNFast + 1>;
using L64 = LiftLaunch<double, 2, kMaxNFast + 1>;

int lift_occupancy_hi(int NP, bool met, bool f64);
int lift_tile_capacity_hi(int NP, bool met, bool f64);
hipError_t launch_lift_hi_f32(const FluxArgs<float> &a, int NP, int grid, bool met, hipStream_t st);
hipError_t launch_lift_hi_f64(const FluxArgs<double> &a, int NP, int grid, bool met, hipStream_t st);

int lift_occupancy(int NP, bool met, bool f64)
{
    if (NP > kMaxNFast + 1) return lift_occupancy_hi(NP, met, f64);
    return f64 ? L64::occupancy(NP, met) : L32::occupancy(NP, met);
}

int lift_tile_capacity(int NP, bool met, bool f64)
{
    if (NP > kMaxNFast + 1) return lift_tile_capacity_hi(NP, met, f64);
    return f64 ? L64::capacity(NP, met) : L32::capacity(NP, met);
}

hipError_t launch_lift_f32(const FluxArgs<float> &a, int NP, int grid, bool met, hipStream_t st)
{
    if (NP > kMaxNFast + 1) return launch_lift_hi_f32(a, NP, grid, met, st);
    return L32::launch(a, NP, grid, met, st);
}

hipError_t launch_lift_f64(const FluxArgs<double> &a, int NP, int grid, bool met, hipStream_t st)
{
    if (NP > kMaxNFast + 1) return launch_lift_hi_f64(a, NP, grid, met, st);
    return L64::launch(a, NP, grid, met, st);
}
#endif

}  // namespace mortar
