// swr_sweep_group.hip -- instantiates the subdomain sweep for a
// time-independent potential with Robin or S0^2 in its shared-factor group
// form: the waves of one workgroup run up to gsize tasks of one factor record
// (the problems of a batch on one subdomain) and read the record from one LDS
// copy, so a wave needs no VGPRs for it and more waves fit on a SIMD.  Used
// for launches that fill the GPU; the arithmetic is the one-wave form's.
#include "swr_sweep_kernel.h"

namespace swr {

template <int P, int TR>
static hipError_t launch_pt(const SweepArgs& a, int gsize, hipStream_t st) {
    const size_t lds = sizeof(cd) * ((size_t)fac_fields(P) * kWave + (size_t)gsize * 2 * kWave) +
                       sizeof(double) * (size_t)gsize * 2 * kWave;
    sweep_kernel<P, TR, VK_STATIC, false, true><<<a.ntasks, gsize * kWave, lds, st>>>(a);
    return hipGetLastError();
}

template <int TR>
static hipError_t launch_t(const SweepArgs& a, int gsize, hipStream_t st) {
    switch (a.P) {
        case 1: return launch_pt<1, TR>(a, gsize, st);
        case 2: return launch_pt<2, TR>(a, gsize, st);
        case 3: return launch_pt<3, TR>(a, gsize, st);
        case 4: return launch_pt<4, TR>(a, gsize, st);
        case 5: return launch_pt<5, TR>(a, gsize, st);
        case 6: return launch_pt<6, TR>(a, gsize, st);
        case 7: return launch_pt<7, TR>(a, gsize, st);
        case 8: return launch_pt<8, TR>(a, gsize, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sweep_groups(const SweepArgs& a, int trans, int gsize, hipStream_t st) {
    if (gsize < 1 || gsize > kGroupMax || !a.groups) return hipErrorInvalidValue;
    if (trans == TR_S02) return launch_t<TR_S02>(a, gsize, st);
    if (trans == TR_ROBIN) return launch_t<TR_ROBIN>(a, gsize, st);
    return hipErrorInvalidValue;
}

}  // namespace swr
