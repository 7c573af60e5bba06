// Instances of the beam-search kernel scoring f32 rows.
#include "fgim_internal.h"

namespace fgim {

hipError_t launch_beam_f32(const BeamArgs& a, bool l2, int nr, int mmax, dim3 grid, size_t smem,
                            hipStream_t s) {
  return l2 ? launch_beam_dispatch<true, kF32>(a, nr, mmax, grid, smem, s)
            : launch_beam_dispatch<false, kF32>(a, nr, mmax, grid, smem, s);
}

}  // namespace fgim
