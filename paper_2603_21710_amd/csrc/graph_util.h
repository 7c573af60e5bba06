// Device helpers shared by the refinement and prune kernels: list keys,
// exclusive scan, CSR construction and the canonical distance between two
// rows read by a group of P lanes.
#pragma once

#include "beam_impl.h"

namespace fgim {

constexpr uint8_t kFlagNew = 1;
constexpr uint8_t kFlagReplaced = 2;
// a list entry (t -> v) that t's Visit recorded, while it was new, as a new
// reverse link of v, not yet consumed by a Visit of v (streamlined rounds)
constexpr uint8_t kFlagRevNew = 4;

// per row of X: squared FP32 norm and squared norm of its BF16 rounding
// residual (round to nearest even)
hipError_t launch_row_norms(const float* X, uint64_t n, uint32_t dim, uint64_t ld, float* nrm2, float* qerr2,
                            hipStream_t s);

// Exclusive scan of n uint32 counts into out[0..n] (out[n] = total).
hipError_t exclusive_scan(const uint32_t* in, uint32_t* out, uint64_t n, uint32_t* block_tmp,
                          hipStream_t s);
uint64_t scan_tmp_words(uint64_t n);

// the P-lane group's chunks of the row at a (sub-lane l holds chunks l,
// l + P, ...; zero where it holds none or when !act)
template <int MMAX>
FGIM_DEV void load_row_chunks(float4 (&x)[MMAX], const float* a, uint32_t nc, int P, int M, int l, bool act) {
#pragma unroll
  for (int mi = 0; mi < MMAX; ++mi) {
    const uint32_t ch = static_cast<uint32_t>(l + mi * P);
    x[mi] = (mi < M && act && ch < nc) ? *reinterpret_cast<const float4*>(a + 4 * ch) : make_float4(0.f, 0.f, 0.f, 0.f);
  }
}

// canonical distance between two rows whose chunks the group holds (as
// load_row_chunks leaves them); every lane of the group gets the result
template <int MMAX>
FGIM_DEV float chunks_distance(const float4 (&x)[MMAX], const float4 (&y)[MMAX], int metric, uint32_t nc, int P, int M,
                               int l, bool act) {
  float s[MMAX];
#pragma unroll
  for (int mi = 0; mi < MMAX; ++mi) {
    s[mi] = 0.0f;
    const uint32_t ch = static_cast<uint32_t>(l + mi * P);
    if (mi < M && act && ch < nc) s[mi] = metric == kL2 ? chunk_sum<kL2>(x[mi], y[mi]) : chunk_sum<kIP>(x[mi], y[mi]);
  }
  return finish_metric(reduce_chunk_sums<MMAX>(s, P, M), metric);
}

// canonical distance between rows a and b (pointers to row starts), computed
// by a group of P lanes (sub-lane l); every lane of the group gets the result
template <int MMAX>
FGIM_DEV float pair_distance(const float* a, const float* b, int metric, uint32_t nc, int P, int M, int l,
                             bool act) {
  float4 x[MMAX], y[MMAX];
  load_row_chunks<MMAX>(x, a, nc, P, M, l, act);
  load_row_chunks<MMAX>(y, b, nc, P, M, l, act);
  return chunks_distance<MMAX>(x, y, metric, nc, P, M, l, act);
}

// canonical distance of the P-lane group's row (chunks held in x) to row
// b, with the loads predicated on `act`; call from wave-uniform code
template <int MMAX>
FGIM_DEV float pair_distance_x(const float4 (&x)[MMAX], const float* b, int metric, uint32_t nc, int P, int M, int l,
                               bool act) {
  float s[MMAX];
#pragma unroll
  for (int mi = 0; mi < MMAX; ++mi) {
    s[mi] = 0.0f;
    const uint32_t ch = static_cast<uint32_t>(l + mi * P);
    if (mi < M && act && ch < nc) {
      const float4 y = *reinterpret_cast<const float4*>(b + 4 * ch);
      s[mi] = metric == kL2 ? chunk_sum<kL2>(x[mi], y) : chunk_sum<kIP>(x[mi], y);
    }
  }
  return finish_metric(reduce_chunk_sums<MMAX>(s, P, M), metric);
}

template <int MMAX>
FGIM_DEV void load_row(float4 (&x)[MMAX], const float* row, uint32_t nc, int P, int M, int l) {
#pragma unroll
  for (int mi = 0; mi < MMAX; ++mi) {
    const uint32_t ch = static_cast<uint32_t>(l + mi * P);
    x[mi] = (mi < M && ch < nc) ? *reinterpret_cast<const float4*>(row + 4 * ch) : make_float4(0.f, 0.f, 0.f, 0.f);
  }
}

// sub-index of global id v given ascending offsets off[0..h)
FGIM_DEV uint32_t sub_of(const uint64_t* off, uint32_t h, uint32_t v) {
  uint32_t lo = 0, hi = h;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) / 2;
    if (v >= off[mid]) lo = mid;
    else hi = mid;
  }
  return lo;
}

}  // namespace fgim
