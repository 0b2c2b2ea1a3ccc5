// swr_sweep_static_pade.hip -- instantiates the subdomain sweep for a
// time-independent potential with the Pade strategy's transmissions
// (S2^{2,m}, S2^{4,m}: m auxiliary functions per interface end, Sec. 2.2).
#include "swr_sweep_kernel.h"

namespace swr {

hipError_t launch_sweep_static_pade(const SweepArgs& a, hipStream_t st) {
    if (!a.endc || !a.pade || a.pade_m < 1 || a.pade_m > kPadeMax) return hipErrorInvalidValue;
    switch (a.P) {
#define CASE(PP)                                                                                 \
    case PP:                                                                                     \
        sweep_kernel<PP, TR_PADE, VK_STATIC><<<a.ntasks, sweep_threads(false), 0, st>>>(a);      \
        break;
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace swr
