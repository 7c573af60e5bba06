// Host-side declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "beam_impl.h"
#include "fgim.h"

namespace fgim {

// beam_{f32,bf16,fp8}.hip: launch the instance matching (l2, nr, mmax)
hipError_t launch_beam_f32(const BeamArgs& a, bool l2, int nr, int mmax, dim3 grid, size_t smem,
                           hipStream_t s);
hipError_t launch_beam_bf16(const BeamArgs& a, bool l2, int nr, int mmax, dim3 grid, size_t smem,
                            hipStream_t s);
hipError_t launch_beam_fp8(const BeamArgs& a, bool l2, int nr, int mmax, dim3 grid, size_t smem,
                           hipStream_t s);

// Launch shape of the beam kernel: P lanes per distance, M = padded chunks /
// P chunks per lane (kernel instance mmax >= M), nr pool registers per lane,
// 2^vis_log2 visited-cache slots, `waves` workgroups (one wave each) per CU.
struct BeamShape {
  uint32_t P, M, mmax, nr, vis_log2, waves;
};

// api.hip: the shape for (dim, L, k), taking every non-zero launch field of
// p as given and the measured defaults for the rest
// mean_degree: the mean out-degree of the graphs searched (0: unknown)
fgim_status beam_shape(uint32_t dim, uint32_t L, uint32_t k, const fgim_params* p, BeamShape* out,
                       double mean_degree = 0.0);
size_t beam_smem(const BeamShape& s);
hipError_t launch_beam(const BeamArgs& a, bool l2, int fmt, const BeamShape& s, hipStream_t st);
// entries of each search re-scored in FP32 in the low-precision forms
fgim_status rerank_for(const fgim_params* p, uint32_t L, uint32_t* out);

// Stage 1 in two parts.  cross_query_check validates the arguments;
// cross_query_run enqueues the beam kernel over buffers the caller provides:
// hdr (4 uint32: queue head, error flag, smallest out-degree, spare), cnt
// (4 counters), subs (device table of h entries) staged from host_subs
// (host, h entries), and the low-precision copy lp / lps when the precision
// is not FP32.  It synchronises the stream before it returns.
struct CrossBufs {
  uint32_t* hdr;
  unsigned long long* cnt;
  SubDev* subs;
  SubDev* host_subs;
  const void* lp;
  const float* lps;
};
fgim_status cross_query_check(const fgim_dataset* d, const fgim_params* p, const uint32_t* ids,
                              const float* dist);
fgim_status cross_query_run(const fgim_dataset* d, const fgim_params* p, uint32_t* ids, float* dist,
                            fgim_stats* stats, hipStream_t s, uint32_t* L_used, const CrossBufs& b);

// prune.hip: neighbour selection over `rows` lists of width k (ids index the
// n_x rows of X; T nullable = no indegree exemption), up to R per list
struct Scratch;
fgim_status select_lists(const float* X, uint64_t n_x, uint64_t ld, uint32_t dim, int metric, uint64_t rows,
                         uint32_t k, uint32_t R, const uint32_t* ids, const float* dist, const uint32_t* T,
                         uint32_t rule, float param, uint32_t flags, const float* nrm2, const float* qerr2,
                         uint32_t* sel_ids, float* sel_dist, uint32_t* sel_n, Scratch& scr, hipStream_t s);

// tune.hip: with a.counter pointing at a zeroed-by-the-callee queue head, a
// graph already validated, and lo the minimum-querying bound on L, choose
// the beam width (*L, lowered only in the batched or low-precision forms) and
// the launch shape; ms_tune gets the time spent on trial launches (0 when
// both came from the cache)
fgim_status tune_stage1(const BeamArgs& a, const fgim_dataset* d, const fgim_params* p, int fmt, bool l2,
                        uint32_t lo, uint32_t* L, BeamShape* shape, double* ms_tune, hipStream_t s);

template <bool L2, int FMT>
hipError_t launch_beam_dispatch(const BeamArgs& a, int nr, int mmax, dim3 grid, size_t smem,
                                hipStream_t s) {
#define FGIM_BEAM_CASE(NR_, MM_)                                                        \
  if (nr == NR_ && mmax == MM_) {                                                       \
    hipLaunchKernelGGL((beam_kernel<L2, FMT, NR_, MM_>), grid, dim3(64), smem, s, a); \
    return hipGetLastError();                                                           \
  }
  FGIM_BEAM_CASE(1, 2)
  FGIM_BEAM_CASE(2, 2)
  FGIM_BEAM_CASE(4, 2)
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
