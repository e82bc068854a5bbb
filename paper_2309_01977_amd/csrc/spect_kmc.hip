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

template <int ATT>
FwdBatchFn fwd_batch_of(bool vec, bool persist)
{
    if (persist) return vec ? fwd_batch<ATT, SPECT_KMC, true, true> : fwd_batch<ATT, SPECT_KMC, false, true>;
    return vec ? fwd_batch<ATT, SPECT_KMC, true, false> : fwd_batch<ATT, SPECT_KMC, false, false>;
}

template <int ATT>
BackBatchFn back_batch_of(bool vec, bool persist)
{
    if (persist) return vec ? back_batch<ATT, SPECT_KMC, true, true> : back_batch<ATT, SPECT_KMC, false, true>;
    return vec ? back_batch<ATT, SPECT_KMC, true, false> : back_batch<ATT, SPECT_KMC, false, false>;
}

FwdBatchFn SPECT_PASTE(fwd_batch_kmc, SPECT_KMC)(int att, bool vec, bool persist)
{
    if (att == ATT_NONE) return fwd_batch_of<ATT_NONE>(vec, persist);
    if (att == ATT_READ) return fwd_batch_of<ATT_READ>(vec, persist);
    return nullptr;
}

BackBatchFn SPECT_PASTE(back_batch_kmc, SPECT_KMC)(int att, bool vec, bool persist)
{
    if (att == ATT_NONE) return back_batch_of<ATT_NONE>(vec, persist);
    if (att == ATT_READ) return back_batch_of<ATT_READ>(vec, persist);
    return nullptr;
}

}  // namespace spectk
