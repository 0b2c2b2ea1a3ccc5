// swr_sweep_cubic_hi.hip -- the subdomain sweep for the |u|^2 potential with
// the W-dependent operators of order 2 and 3 (S0^3, S1^2, S2^{2,m}; W_n =
// |v_{n-1}|^2 at the end node, refactorised every step): dispatch on the chunk
// width to swr_sweep_cubic_hi_p1.hip .. swr_sweep_cubic_hi_p8.hip.
#include "swr_common.h"

namespace swr {

template <int P>
void launch_sweep_cubic_hi_p(const SweepArgs& a, int trans, hipStream_t st);

hipError_t launch_sweep_cubic_hi(const SweepArgs& a, int trans, hipStream_t st) {
    if (trans != TR_GEN && trans != TR_PADE) return hipErrorInvalidValue;
    if (trans == TR_GEN && !a.endc) return hipErrorInvalidValue;
    if (trans == TR_PADE && (!a.pade || a.pade_m < 1 || a.pade_m > kPadeMax || a.pade_order != 2))
        return hipErrorInvalidValue;
    // the order-4 operators carry dn f(u): not provided
    if (a.tr == 3 || a.tr == 5 || a.tr == 7) return hipErrorInvalidValue;
    switch (a.P) {
        case 1: launch_sweep_cubic_hi_p<1>(a, trans, st); break;
        case 2: launch_sweep_cubic_hi_p<2>(a, trans, st); break;
        case 3: launch_sweep_cubic_hi_p<3>(a, trans, st); break;
        case 4: launch_sweep_cubic_hi_p<4>(a, trans, st); break;
        case 5: launch_sweep_cubic_hi_p<5>(a, trans, st); break;
        case 6: launch_sweep_cubic_hi_p<6>(a, trans, st); break;
        case 7: launch_sweep_cubic_hi_p<7>(a, trans, st); break;
        case 8: launch_sweep_cubic_hi_p<8>(a, trans, st); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace swr
