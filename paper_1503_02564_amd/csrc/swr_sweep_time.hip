// swr_sweep_time.hip -- the subdomain sweep for a time-dependent potential
// V(t,x): dispatch on the chunk width P to the instantiations in
// swr_sweep_time_p1.hip .. swr_sweep_time_p8.hip (Robin, S0^2) and
// swr_sweep_time_hi_p1.hip .. swr_sweep_time_hi_p8.hip (higher-order and Pade).
#include "swr_common.h"

namespace swr {

template <int P>
hipError_t launch_sweep_time_p(const SweepArgs& a, int trans, hipStream_t st);
template <int P>
hipError_t launch_sweep_time_hi_p(const SweepArgs& a, int trans, hipStream_t st);

hipError_t launch_sweep_time(const SweepArgs& a, int trans, hipStream_t st) {
    if (trans == TR_GEN || trans == TR_PADE) {
        // higher-order and Pade operators (swr_sweep_time_hi_p*.hip)
        if (trans == TR_GEN && !a.endc) return hipErrorInvalidValue;
        if (trans == TR_PADE && (!a.pade || a.pade_m < 1 || a.pade_m > kPadeMax)) return hipErrorInvalidValue;
        switch (a.P) {
            case 1: return launch_sweep_time_hi_p<1>(a, trans, st);
            case 2: return launch_sweep_time_hi_p<2>(a, trans, st);
            case 3: return launch_sweep_time_hi_p<3>(a, trans, st);
            case 4: return launch_sweep_time_hi_p<4>(a, trans, st);
            case 5: return launch_sweep_time_hi_p<5>(a, trans, st);
            case 6: return launch_sweep_time_hi_p<6>(a, trans, st);
            case 7: return launch_sweep_time_hi_p<7>(a, trans, st);
            case 8: return launch_sweep_time_hi_p<8>(a, trans, st);
            default: return hipErrorInvalidValue;
        }
    }
    if (trans != TR_S02 && trans != TR_ROBIN) return hipErrorInvalidValue;
    switch (a.P) {
        case 1: return launch_sweep_time_p<1>(a, trans, st);
        case 2: return launch_sweep_time_p<2>(a, trans, st);
        case 3: return launch_sweep_time_p<3>(a, trans, st);
        case 4: return launch_sweep_time_p<4>(a, trans, st);
        case 5: return launch_sweep_time_p<5>(a, trans, st);
        case 6: return launch_sweep_time_p<6>(a, trans, st);
        case 7: return launch_sweep_time_p<7>(a, trans, st);
        case 8: return launch_sweep_time_p<8>(a, trans, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace swr
