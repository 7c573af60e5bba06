// Device-side building blocks of the FGIM kernels for gfx950 (CDNA4,
// 64-lane wavefronts).
//
// Ordering keys.  Every list is ordered by (delta, id).  A key packs both in
// a uint64: the high word is the FP32 bit pattern mapped to an unsigned
// integer with the same order (flip all bits of negatives, set the sign bit
// of non-negatives), the low word is the id.  Integer comparison of keys is
// then the (delta ascending, id ascending) total order.  kSentinel (all
// ones) sorts after every real key and marks an empty slot.
//
// Canonical distance.  The d coordinates form nc = d/4 chunks, padded with
// zero chunks to N = 2^ceil(log2 nc).  A chunk is summed with four fused
// multiply-adds from +0; the chunk sums are combined by the stride tree
// s[c] += s[c + st] for st = N/2 ... 1.  With P lanes per distance (P a
// power of two <= N), lane l owns chunks l, l+P, ... (M = N/P of them): the
// strides >= P combine chunks of one lane and run in registers, the strides
// < P run as xor butterflies across the P lanes.  Because FP32 addition is
// commutative, every lane of the group ends with the same bits, and those
// bits do not depend on P.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define FGIM_DEV __device__ __forceinline__

namespace fgim {

constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr uint64_t kSentinel = ~0ull;
constexpr int kWave = 64;

enum Metric : int { kL2 = 0, kIP = 1, kCos = 2 };

FGIM_DEV uint32_t order_bits(float d) {
  uint32_t u = __float_as_uint(d);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

FGIM_DEV float bits_to_dist(uint32_t o) {
  uint32_t u = (o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o;
  return __uint_as_float(u);
}

FGIM_DEV uint64_t make_key(float d, uint32_t id) {
  return (static_cast<uint64_t>(order_bits(d)) << 32) | id;
}

FGIM_DEV uint32_t key_id(uint64_t k) { return static_cast<uint32_t>(k); }

FGIM_DEV float key_dist(uint64_t k) {
  return k == kSentinel ? __builtin_inff() : bits_to_dist(static_cast<uint32_t>(k >> 32));
}

FGIM_DEV int lane_id() { return __lane_id(); }

FGIM_DEV uint64_t ballot(bool p) { return __ballot(p); }

FGIM_DEV int popc64(uint64_t m) { return __popcll(m); }

// index of the lowest set bit of a non-zero mask
FGIM_DEV int ffs64(uint64_t m) { return __ffsll(static_cast<unsigned long long>(m)) - 1; }

// number of set bits of m below this lane
FGIM_DEV int mbcnt(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(m >> 32),
                                   __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(m), 0));
}

FGIM_DEV uint32_t readlane(uint32_t v, int l) { return __builtin_amdgcn_readlane(v, l); }

FGIM_DEV uint64_t readlane64(uint64_t v, int l) {
  uint32_t lo = __builtin_amdgcn_readlane(static_cast<uint32_t>(v), l);
  uint32_t hi = __builtin_amdgcn_readlane(static_cast<uint32_t>(v >> 32), l);
  return (static_cast<uint64_t>(hi) << 32) | lo;
}

FGIM_DEV uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// orders this wavefront's LDS writes before its later LDS reads (lanes of
// one wavefront exchanging data through LDS)
FGIM_DEV void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

FGIM_DEV float shfl_xor_f(float v, int m) { return __shfl_xor(v, m, kWave); }

FGIM_DEV uint32_t shfl_u(uint32_t v, int src) { return __shfl(v, src, kWave); }

FGIM_DEV uint64_t shfl64(uint64_t v, int src) {
  uint32_t lo = __shfl(static_cast<uint32_t>(v), src, kWave);
  uint32_t hi = __shfl(static_cast<uint32_t>(v >> 32), src, kWave);
  return (static_cast<uint64_t>(hi) << 32) | lo;
}

// lane i receives lane i-1's value; lane 0 receives `first`
FGIM_DEV uint64_t shift_up64(uint64_t v, uint64_t first) {
  uint64_t up = shfl64(v, lane_id() == 0 ? 0 : lane_id() - 1);
  return lane_id() == 0 ? first : up;
}

FGIM_DEV uint32_t shift_up32(uint32_t v, uint32_t first) {
  uint32_t up = shfl_u(v, lane_id() == 0 ? 0 : lane_id() - 1);
  return lane_id() == 0 ? first : up;
}

// ---------------------------------------------------------------------------
// chunk arithmetic (4 coordinates)

template <int METRIC>
FGIM_DEV float chunk_sum(const float4 q, const float4 x) {
  float s = 0.0f;
  if (METRIC == kL2) {
    float e0 = q.x - x.x, e1 = q.y - x.y, e2 = q.z - x.z, e3 = q.w - x.w;
    s = __builtin_fmaf(e0, e0, s);
    s = __builtin_fmaf(e1, e1, s);
    s = __builtin_fmaf(e2, e2, s);
    s = __builtin_fmaf(e3, e3, s);
  } else {
    s = __builtin_fmaf(q.x, x.x, s);
    s = __builtin_fmaf(q.y, x.y, s);
    s = __builtin_fmaf(q.z, x.z, s);
    s = __builtin_fmaf(q.w, x.w, s);
  }
  return s;
}

template <int METRIC>
FGIM_DEV float finish(float r) {
  float d = METRIC == kL2 ? r : (METRIC == kIP ? -r : 1.0f - r);
  return d + 0.0f;
}

FGIM_DEV float finish_metric(float r, int metric) {
  if (metric == kL2) return finish<kL2>(r);
  if (metric == kIP) return finish<kIP>(r);
  return finish<kCos>(r);
}

// The canonical order's reduction inside a group of P lanes (P a power of
// two): s[mi] holds the sum of the lane's chunk l + mi * P, or zero where the
// lane holds none, for the first M (a power of two) of MMAX entries.  The
// stride tree s[c] += s[c + st] over the zero-padded chunks runs in
// registers for strides >= P (the lane's own entries) and as xor
// butterflies for strides < P, so every lane of the group ends with the
// same bits for any P.  Every distance of the library goes through here.
template <int MMAX>
FGIM_DEV float reduce_chunk_sums(float (&s)[MMAX], int P, int M) {
#pragma unroll
  for (int st = MMAX / 2; st >= 1; st /= 2) {
    if (2 * st <= M) {
#pragma unroll
      for (int i = 0; i < st; ++i) s[i] = s[i] + s[i + st];
    }
  }
  float r = s[0];
#pragma unroll
  for (int st = 32; st >= 1; st /= 2)
    if (st < P) r = r + shfl_xor_f(r, st);
  return r;
}

// ---------------------------------------------------------------------------
// row formats

// A row format gives raw(row, c): the stored bytes of chunk c (4 values),
// scale(row): the row's factor (1 when the format has none), and
// decode(raw, scale): the chunk as FP32.  chunk() is both at once.  Loads of
// raw chunks are cheap on registers, so a scorer can keep more in flight.
struct RowF32 {
  typedef float4 Raw;
  const float* base;
  uint64_t ld;
  FGIM_DEV Raw raw(uint64_t row, uint32_t c) const {
    return *reinterpret_cast<const float4*>(base + row * ld + 4ull * c);
  }
  FGIM_DEV float scale(uint64_t) const { return 1.0f; }
  FGIM_DEV static float4 decode(Raw v, float) { return v; }
  FGIM_DEV float4 chunk(uint64_t row, uint32_t c) const { return raw(row, c); }
};

struct RowBF16 {
  typedef uint2 Raw;
  const uint16_t* base;  // dense rows of `dim`
  uint32_t dim;
  FGIM_DEV Raw raw(uint64_t row, uint32_t c) const {
    return *reinterpret_cast<const uint2*>(base + row * dim + 4ull * c);
  }
  FGIM_DEV float scale(uint64_t) const { return 1.0f; }
  FGIM_DEV static float4 decode(Raw v, float) {
    float4 f;
    f.x = __uint_as_float(v.x << 16);
    f.y = __uint_as_float(v.x & 0xFFFF0000u);
    f.z = __uint_as_float(v.y << 16);
    f.w = __uint_as_float(v.y & 0xFFFF0000u);
    return f;
  }
  FGIM_DEV float4 chunk(uint64_t row, uint32_t c) const { return decode(raw(row, c), 1.0f); }
};

struct RowFP8 {
  typedef uint32_t Raw;
  const uint8_t* base;  // dense rows of `dim`
  const float* scales;
  uint32_t dim;
  FGIM_DEV Raw raw(uint64_t row, uint32_t c) const {
    return *reinterpret_cast<const uint32_t*>(base + row * dim + 4ull * c);
  }
  FGIM_DEV float scale(uint64_t row) const { return scales[row]; }
  // OCP E4M3 ("fn": bias 7, no infinities); gfx950's packed conversion reads
  // this format and is exact
  FGIM_DEV static float4 decode(Raw v, float s) {
    const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8(static_cast<int>(v), false);
    const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8(static_cast<int>(v), true);
    float4 f;
    f.x = s * lo[0];
    f.y = s * lo[1];
    f.z = s * hi[0];
    f.w = s * hi[1];
    return f;
  }
  FGIM_DEV float4 chunk(uint64_t row, uint32_t c) const { return decode(raw(row, c), scale(row)); }
};

}  // namespace fgim
