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

KernelFn SPECT_PASTE(fwd_kernel_kmc, SPECT_KMC)(int att, bool vec)
{
    switch (att) {
    case ATT_NONE: return vec ? fwd_main<ATT_NONE, SPECT_KMC, true> : fwd_main<ATT_NONE, SPECT_KMC, false>;
    case ATT_SAMPLE: return vec ? fwd_main<ATT_SAMPLE, SPECT_KMC, true> : fwd_main<ATT_SAMPLE, SPECT_KMC, false>;
    case ATT_READ: return vec ? fwd_main<ATT_READ, SPECT_KMC, true> : fwd_main<ATT_READ, SPECT_KMC, false>;
    default: return nullptr;
    }
}

BackFn SPECT_PASTE(back_kernel_kmc, SPECT_KMC)(int att, bool vec)
{
    switch (att) {
    case ATT_NONE: return vec ? back_rot<ATT_NONE, SPECT_KMC, true> : back_rot<ATT_NONE, SPECT_KMC, false>;
    case ATT_SAMPLE: return vec ? back_rot<ATT_SAMPLE, SPECT_KMC, true> : back_rot<ATT_SAMPLE, SPECT_KMC, false>;
    case ATT_WRITE: return vec ? back_rot<ATT_WRITE, SPECT_KMC, true> : back_rot<ATT_WRITE, SPECT_KMC, false>;
    case ATT_READ: return vec ? back_rot<ATT_READ, SPECT_KMC, true> : back_rot<ATT_READ, SPECT_KMC, false>;
    default: return nullptr;
    }
}

}  // namespace spectk
