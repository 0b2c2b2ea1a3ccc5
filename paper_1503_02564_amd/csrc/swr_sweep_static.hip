// swr_sweep_static.hip -- instantiates the subdomain sweep for a time-independent
// potential with the Robin and higher-order transmissions (S0^2 is in
// swr_sweep_static_s02.hip, the Pade strategy in swr_sweep_static_pade.hip).
#include "swr_sweep_kernel.h"

namespace swr {

template <int P>
static void launch_p(const SweepArgs& a, int trans, hipStream_t st) {
    if (trans == TR_GEN) sweep_kernel<P, TR_GEN, VK_STATIC><<<a.ntasks, sweep_threads(false), 0, st>>>(a);
    else sweep_kernel<P, TR_ROBIN, VK_STATIC><<<a.ntasks, sweep_threads(false), 0, st>>>(a);
}

hipError_t launch_sweep_static(const SweepArgs& a, int trans, hipStream_t st) {
    if (trans == TR_S02) return launch_sweep_static_s02(a, st);
    if (trans == TR_PADE) return launch_sweep_static_pade(a, st);
    if (trans == TR_GEN && !a.endc) return hipErrorInvalidValue;
    switch (a.P) {
        case 1: launch_p<1>(a, trans, st); break;
        case 2: launch_p<2>(a, trans, st); break;
        case 3: launch_p<3>(a, trans, st); break;
        case 4: launch_p<4>(a, trans, st); break;
        case 5: launch_p<5>(a, trans, st); break;
        case 6: launch_p<6>(a, trans, st); break;
        case 7: launch_p<7>(a, trans, st); break;
        case 8: launch_p<8>(a, trans, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace swr
