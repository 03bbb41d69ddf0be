// Fixed device scratch of the allocation-free volume update (rbf_volume_update_noalloc): the
// reduced-point list, the per-block counts and the split partial sums of the plain volume update
// live in this array instead of pool memory. It is part of the library's code object, so each
// device the library runs on holds its own copy until the process ends. Host code must use the
// address hipGetSymbolAddress returns for the current device, never the array's name.
#include "internal.h"

namespace rbf {

static __device__ __align__(256) unsigned char scratch[RBF_NOALLOC_SCRATCH_BYTES];

rbf_status noalloc_scratch_address(void **ptr)
{
    *ptr = nullptr;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(RBF_E_DEVICE, "hipGetSymbolAddress of the fixed scratch failed: %s", hipGetErrorString(e));
    *ptr = p;
    return RBF_OK;
}

}  // namespace rbf
