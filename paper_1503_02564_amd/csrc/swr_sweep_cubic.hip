// swr_sweep_cubic.hip -- instantiates the subdomain sweep for the |u|^2 potential
// (Robin and S0^2; the W-dependent operators are in swr_sweep_cubic_hi.hip).
#include "swr_sweep_kernel.h"

namespace swr {

template <int P>
static void launch_p(const SweepArgs& a, int trans, hipStream_t st) {
    if (trans == TR_S02 && a.ntasks <= a.help_max)
        sweep_kernel<P, TR_S02, VK_CUBIC, true><<<a.ntasks, sweep_threads(true), 0, st>>>(a);
    else if (trans == TR_S02)
        sweep_kernel<P, TR_S02, VK_CUBIC, false><<<a.ntasks, sweep_threads(false), 0, st>>>(a);
    else sweep_kernel<P, TR_ROBIN, VK_CUBIC><<<a.ntasks, sweep_threads(false), 0, st>>>(a);
}

hipError_t launch_sweep_cubic_hi(const SweepArgs& a, int trans, hipStream_t st);

hipError_t launch_sweep_cubic(const SweepArgs& a, int trans, hipStream_t st) {
    // the W-dependent operators (swr_sweep_cubic_hi.hip)
    if (trans == TR_GEN || trans == TR_PADE) return launch_sweep_cubic_hi(a, trans, st);
    if (trans != TR_S02 && trans != TR_ROBIN) return hipErrorInvalidValue;
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
