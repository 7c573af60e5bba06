// Entry points of stages 2 and 3 until their kernels land.
#include "host_util.h"

extern "C" {

fgim_status fgim_refine(const fgim_dataset*, const fgim_params*, uint32_t*, float*, uint32_t*, fgim_stats*,
                        void*) {
  return fgim::fail(FGIM_ERR_UNSUPPORTED, "fgim_refine is not built yet");
}

fgim_status fgim_prune(const fgim_dataset*, const fgim_params*, const uint32_t*, const float*, const uint32_t*,
                       uint32_t*, uint32_t*, void*) {
  return fgim::fail(FGIM_ERR_UNSUPPORTED, "fgim_prune is not built yet");
}

fgim_status fgim_merge(const fgim_dataset*, const fgim_params*, uint32_t*, uint32_t*, uint32_t*, fgim_stats*,
                       void*) {
  return fgim::fail(FGIM_ERR_UNSUPPORTED, "fgim_merge is not built yet");
}

}  // extern "C"
