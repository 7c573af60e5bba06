// Host-side declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "beam_impl.h"

namespace fgim {

// beam_{f32,bf16,fp8}.hip: launch the instance matching (l2, nr, mmax)
hipError_t launch_beam_f32(const BeamArgs& a, bool l2, int nr, int mmax, dim3 grid, size_t smem,
                           hipStream_t s);
hipError_t launch_beam_bf16(const BeamArgs& a, bool l2, int nr, int mmax, dim3 grid, size_t smem,
                            hipStream_t s);
hipError_t launch_beam_fp8(const BeamArgs& a, bool l2, int nr, int mmax, dim3 grid, size_t smem,
                           hipStream_t s);

template <bool L2, int FMT>
hipError_t launch_beam_dispatch(const BeamArgs& a, int nr, int mmax, dim3 grid, size_t smem,
                                hipStream_t s) {
#define FGIM_BEAM_CASE(NR_, MM_)                                                        \
  if (nr == NR_ && mmax == MM_) {                                                       \
    hipLaunchKernelGGL((beam_kernel<L2, FMT, NR_, MM_>), grid, dim3(64), smem, s, a); \
    return hipGetLastError();                                                           \
  }
  FGIM_BEAM_CASE(1, 4)
  FGIM_BEAM_CASE(2, 4)
  FGIM_BEAM_CASE(4, 4)
  FGIM_BEAM_CASE(1, 16)
  FGIM_BEAM_CASE(2, 16)
  FGIM_BEAM_CASE(4, 16)
#undef FGIM_BEAM_CASE
  return hipErrorInvalidValue;
}

}  // namespace fgim
