// Per-device static scratch of chimera_lnl_batch_static (library-internal):
// the device memory that entry point lays its per-call buffers out in, so
// that it allocates nothing.  One copy of the array per GPU, held from the
// library's load until the process ends.
#include <hip/hip_runtime.h>

#include "launch.h"

namespace chimera {

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

// The device address of the current device's copy of `scratch` (host code
// must use this address, never the array's name).
hipError_t static_scratch_address(void** ptr) {
  return hipGetSymbolAddress(ptr, HIP_SYMBOL(scratch));
}

}  // namespace chimera
