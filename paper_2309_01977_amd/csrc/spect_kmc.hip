// spect_kmc.hip - the forward and rotated-frame back-projection kernels of
// one blur-radius class, compiled once per class with -DSPECT_KMC=<class>
// (0, 4, ..., 32) so that the classes build in parallel.
#include "spect_device.h"

#ifndef SPECT_KMC
#error "compile with -DSPECT_KMC=<blur radius class>"
#endif

#define SPECT_PASTE2(a, b) a##b
#define SPECT_PASTE(a, b) SPECT_PASTE2(a, b)

namespace spectk {

KernelFn SPECT_PASTE(fwd_kernel_kmc, SPECT_KMC)(bool mu, bool vec)
{
    if (mu) return vec ? fwd_main<true, SPECT_KMC, true> : fwd_main<true, SPECT_KMC, false>;
    return vec ? fwd_main<false, SPECT_KMC, true> : fwd_main<false, SPECT_KMC, false>;
}

BackFn SPECT_PASTE(back_kernel_kmc, SPECT_KMC)(bool mu, bool vec)
{
    if (mu) return vec ? back_rot<true, SPECT_KMC, true> : back_rot<true, SPECT_KMC, false>;
    return vec ? back_rot<false, SPECT_KMC, true> : back_rot<false, SPECT_KMC, false>;
}

}  // namespace spectk
