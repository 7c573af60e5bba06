// Instances of the beam-search kernel scoring fp8 rows.
#include "fgim_internal.h"

namespace fgim {

hipError_t launch_beam_fp8(const BeamArgs& a, bool l2, int nr, int mmax, dim3 grid, size_t smem,
                            hipStream_t s) {
  return l2 ? launch_beam_dispatch<true, kFP8>(a, nr, mmax, grid, smem, s)
            : launch_beam_dispatch<false, kFP8>(a, nr, mmax, grid, smem, s);
}

}  // namespace fgim
