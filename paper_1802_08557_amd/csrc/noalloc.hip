// noalloc.hip -- the device scratch of lp_batch_solve_noalloc, the solve entry
// point for callers that cannot allocate device memory.
//
// The array below is statically allocated in the library's code object: every
// device the library runs on holds its own copy from the moment the code
// object is loaded there until the process ends.  Host code never uses the
// array's name as an address -- on the host it names a stand-in, not device
// memory -- but the device address that hipGetSymbolAddress returns for the
// current device, looked up once per context (lp_ctx_create) and kept there.
//
// Layout (internal.h, kNoAlloc*): work counters in the first 256 bytes, then
// the list of LPs the wavefront kernel defers (kNoAllocMaxLps int32), then the
// workgroup kernel's tableau slots for those LPs.  Every call on a device
// shares the one array, so calls that overlap on a device race.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace lpb {

static __device__ __align__(256) char scratch[kNoAllocBytes];

hipError_t noalloc_scratch_address(void **ptr)
{
    *ptr = nullptr;
    return hipGetSymbolAddress(ptr, HIP_SYMBOL(scratch));
}

}  // namespace lpb
