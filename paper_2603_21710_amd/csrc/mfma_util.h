// BF16 operands for v_mfma_f32_16x16x32_bf16 and the rigorous error bound of
// a BF16 inner product, shared by the MFMA join and the MFMA neighbour
// selection.  Both screen pairs on MFMA and re-score in canonical FP32 only
// the pairs the bound cannot decide, so their results equal the plain FP32
// computation bit for bit.
#pragma once

#include "fgim_device.h"

namespace fgim {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef short shortx8_t __attribute__((ext_vector_type(8)));
typedef float floatx4_t __attribute__((ext_vector_type(4)));

// x rounded to BF16 (nearest even), as FP32
FGIM_DEV float bf16_value(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xFFFF0000u);
}

// x rounded to BF16 (nearest even), as bits
FGIM_DEV uint16_t bf16_rne(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}

// gamma = (d + 4) u / (1 - (d + 4) u), u = 2^-24: the relative bound of an
// FP32 sum of d + 4 terms in any order
FGIM_DEV float fp32_gamma(uint32_t dim) {
  const float u32 = 5.9604645e-8f;
  return (dim + 4) * u32 / (1.0f - (dim + 4) * u32);
}

// Distance estimate dt from the MFMA inner product G of the BF16 operands
// a^, b^, and a bound err with |dt - delta| <= err for the canonical FP32
// distance delta of (a, b).  na2, nb2: squared FP32 norms; ea, eb: BF16
// residual norms |a - a^|, |b - b^| inflated by their own rounding bound.
//   |<a^,b^>_mfma - <a,b>| <= e_a (|b| + e_b) + |a| e_b + gamma (|a| + e_a)(|b| + e_b)
// (Cauchy-Schwarz on the residuals plus any-order FP32 accumulation); the L2
// estimate adds the FP32 norms' own error, and the canonical distance is
// within gamma of the true value.  The bound returned is doubled.
FGIM_DEV void screen_estimate(float G, float na2, float nb2, float ea, float eb, float gam, int metric, float* dt,
                              float* err) {
  const float u32 = 5.9604645e-8f;
  const float na = sqrtf(na2) * (1.0f + gam) * 1.0001f, nb = sqrtf(nb2) * (1.0f + gam) * 1.0001f;
  const float eg = ea * (nb + eb) + na * eb + gam * (na + ea) * (nb + eb) + 1e-30f;
  float d, e;
  if (metric == kL2) {
    d = na2 + nb2 - 2.0f * G;
    e = gam * (na2 + nb2) + 2.0f * eg + 4.0f * u32 * (na2 + nb2 + 2.0f * fabsf(G));
    e += gam * (fabsf(d) + e);
  } else if (metric == kIP) {
    d = -G;
    e = eg + gam * na * nb;
  } else {
    d = 1.0f - G;
    e = eg + gam * na * nb + u32 * (1.0f + fabsf(G));
  }
  *dt = d;
  *err = 2.0f * e;
}

}  // namespace fgim
