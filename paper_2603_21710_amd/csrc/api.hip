// C ABI of libfgim: argument validation, the scratch arena, launch
// shape selection and the small utility kernels (graph validation, fills,
// low-precision encoders).  The stage kernels live in beam_*.hip,
// refine.hip and prune.hip.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "fgim.h"
#include "fgim_internal.h"
#include "host_util.h"

namespace fgim {

thread_local std::string g_last_error;

fgim_status fail(fgim_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

void clear_error() { g_last_error.clear(); }

int device_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
    return 256;
  return cus;
}

hipError_t library_stream(hipStream_t* out) {
  static hipStream_t streams[64] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  static std::mutex mu;
  std::lock_guard<std::mutex> lock(mu);
  if (!streams[dev]) {
    e = hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking);
    if (e != hipSuccess) return e;
  }
  *out = streams[dev];
  return hipSuccess;
}

void keep_scratch_cached() {
  static std::once_flag once[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
    (void)hipGetLastError();
    return;
  }
  std::call_once(once[dev], [dev] {
    hipMemPool_t pool = nullptr;
    uint64_t cur = 0;
    if (hipDeviceGetMemPool(&pool, dev) == hipSuccess && pool &&
        hipMemPoolGetAttribute(pool, hipMemPoolAttrReleaseThreshold, &cur) == hipSuccess && cur == 0) {
      uint64_t keep = ~0ull;
      (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
    (void)hipGetLastError();
  });
}

namespace {

struct Arena {
  std::recursive_mutex mu;
  char* base = nullptr;
  size_t cap = 0;   // bytes at base
  size_t top = 0;   // bytes taken by the live scopes
  size_t virt = 0;  // bytes the live scopes asked for, spilled ones included
  size_t high = 0;  // the largest virt seen: the size the next growth aims at
  int depth = 0;    // live scopes
  hipEvent_t done = nullptr;
  bool pending = false;  // done marks the last call's device work
};

Arena g_arena[64];
constexpr size_t kArenaAlign = 256;

size_t arena_align(size_t x) { return (x + kArenaAlign - 1) & ~(kArenaAlign - 1); }

}  // namespace

Scratch::Scratch(hipStream_t st) : s(st) {
  keep_scratch_cached();
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
    (void)hipGetLastError();
    dev = -1;
    return;
  }
  Arena& a = g_arena[dev];
  a.mu.lock();
  if (a.depth == 0) {
    if (a.pending) (void)hipStreamWaitEvent(s, a.done, 0);
    if (a.high > a.cap) {
      // the last call's device work may still use the old buffer
      if (a.pending) (void)hipEventSynchronize(a.done);
      if (a.base) (void)hipFree(a.base);
      a.base = nullptr;
      a.cap = 0;
      const size_t want = arena_align(a.high + a.high / 8);
      if (hipMalloc(&a.base, want) == hipSuccess && a.base) a.cap = want;
      else a.base = nullptr;
    }
    (void)hipGetLastError();
    a.top = 0;
    a.virt = 0;
  }
  mark_top = a.top;
  mark_virt = a.virt;
  ++a.depth;
}

void* Scratch::take(size_t bytes) {
  if (dev < 0) return nullptr;
  Arena& a = g_arena[dev];
  const size_t b = arena_align(bytes);
  a.virt += b;
  a.high = std::max(a.high, a.virt);
  if (a.top + b > a.cap) return nullptr;
  void* p = a.base + a.top;
  a.top += b;
  return p;
}

Scratch::~Scratch() {
  for (void* p : spill) (void)hipFreeAsync(p, s);
  if (dev < 0) return;
  Arena& a = g_arena[dev];
  a.top = mark_top;
  a.virt = mark_virt;
  if (--a.depth == 0) {
    if (!a.done && hipEventCreateWithFlags(&a.done, hipEventDisableTiming) != hipSuccess) a.done = nullptr;
    a.pending = a.done && hipEventRecord(a.done, s) == hipSuccess;
    (void)hipGetLastError();
  }
  a.mu.unlock();
}

fgim_status release_scratch() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
    (void)hipGetLastError();
    return fail(FGIM_ERR_DEVICE, "no current HIP device");
  }
  Arena& a = g_arena[dev];
  std::lock_guard<std::recursive_mutex> lock(a.mu);
  if (a.depth) return fail(FGIM_ERR_INVALID_ARG, "scratch is in use by a call on this thread");
  if (a.pending) HIP_TRY(hipEventSynchronize(a.done));
  a.pending = false;
  if (a.base) HIP_TRY(hipFree(a.base));
  a.base = nullptr;
  a.cap = 0;
  a.high = 0;
  return FGIM_OK;
}

// ---------------------------------------------------------------------------
// utility kernels

__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, uint64_t n) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    p[i] = v;
}

hipError_t fill_u32(uint32_t* p, uint32_t v, uint64_t n, hipStream_t s) {
  if (n == 0) return hipSuccess;
  uint64_t blocks = std::min<uint64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(fill_u32_kernel, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

// One wavefront per adjacency row: every id must be FGIM_NONE or < n, not
// the row's own id, and unique within the row.  Sets *err on a violation;
// when min_deg is given, lowers *min_deg to the smallest out-degree seen, and
// when edges is given, adds the sum of the out-degrees times `weight` to
// *edges.
__global__ void __launch_bounds__(256) validate_graph_kernel(const uint32_t* adj, uint32_t n,
                                                             uint32_t stride, uint32_t* err,
                                                             uint32_t* min_deg, double* edges, double weight) {
  const uint32_t wave = threadIdx.x / 64;
  const int lane = lane_id();
  uint32_t mdeg = 0xFFFFFFFFu;
  unsigned long long esum = 0;
  for (uint64_t row = blockIdx.x * 4ull + wave; row < n; row += gridDim.x * 4ull) {
    const uint32_t v0 = lane < static_cast<int>(stride) ? adj[row * stride + lane] : kNone;
    const uint32_t v1 = lane + 64 < static_cast<int>(stride) ? adj[row * stride + 64 + lane] : kNone;
    const uint32_t deg = static_cast<uint32_t>(popc64(ballot(v0 != kNone)) + popc64(ballot(v1 != kNone)));
    mdeg = deg < mdeg ? deg : mdeg;
    esum += deg;
    bool bad = (v0 != kNone && (v0 >= n || v0 == row)) || (v1 != kNone && (v1 >= n || v1 == row));
    for (int s = 1; s < 64; ++s) {
      const uint32_t w0 = __shfl_xor(v0, s, 64);
      bad |= v0 != kNone && w0 == v0;
      if (stride > 64) {
        const uint32_t w1 = __shfl_xor(v1, s, 64);
        bad |= v1 != kNone && w1 == v1;
      }
    }
    if (stride > 64) {
      for (int s = 0; s < 64; ++s) {
        const uint32_t w1 = __shfl(v1, s, 64);
        bad |= v0 != kNone && w1 == v0;
      }
    }
    if (ballot(bad) != 0 && lane == 0) atomicOr(err, 1u);
  }
  if (min_deg && lane == 0 && mdeg != 0xFFFFFFFFu) atomicMin(min_deg, mdeg);
  // one atomic per workgroup: every wave adding to the one counter would
  // serialise thousands of device-scope atomics
  __shared__ unsigned long long s_e[4];
  if (lane == 0) s_e[wave] = esum;
  __syncthreads();
  if (edges && threadIdx.x == 0) {
    const unsigned long long t = s_e[0] + s_e[1] + s_e[2] + s_e[3];
    if (t) atomicAdd(edges, static_cast<double>(t) * weight);
  }
}

hipError_t validate_graph(const uint32_t* adj, uint32_t n, uint32_t stride, uint32_t* err,
                          hipStream_t s, uint32_t* min_deg = nullptr, double* edges = nullptr,
                          double weight = 1.0) {
  uint32_t blocks = std::min<uint32_t>((n + 3) / 4, 2048);
  hipLaunchKernelGGL(validate_graph_kernel, dim3(blocks), dim3(256), 0, s, adj, n, stride, err, min_deg, edges,
                     weight);
  return hipGetLastError();
}

// BF16: round to nearest even (NaN stays a quiet NaN).
__device__ __forceinline__ uint16_t bf16_encode(float x) {
  uint32_t u = __float_as_uint(x);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) return static_cast<uint16_t>((u >> 16) | 0x40u);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return static_cast<uint16_t>(u >> 16);
}

// OCP E4M3, round to nearest even, saturating at 448.  Below 2^-6 the code
// is the subnormal mantissa round(|x| * 2^9) (8 carries into the smallest
// normal, code 0x08); above, the FP32 mantissa is cut to 3 bits with
// round-half-even on the 20 dropped bits.
__device__ __forceinline__ uint8_t fp8_encode(float x) {
  const uint32_t bits = __float_as_uint(x);
  const uint32_t sign = (bits >> 24) & 0x80u;
  const float a = __uint_as_float(bits & 0x7FFFFFFFu);
  if (!(a < 448.0f)) return static_cast<uint8_t>(sign | 0x7Eu);
  if (a < 0.015625f) {
    const uint32_t m = static_cast<uint32_t>(__builtin_rintf(a * 512.0f));
    return static_cast<uint8_t>(sign | m);
  }
  const uint32_t ab = bits & 0x7FFFFFFFu;
  int e = static_cast<int>(ab >> 23) - 127;
  const uint32_t mant = ab & 0x7FFFFFu;
  uint32_t r = mant >> 20;
  const uint32_t rem = mant & 0xFFFFFu;
  if (rem > 0x80000u || (rem == 0x80000u && (r & 1u))) ++r;
  if (r == 8u) {
    r = 0;
    ++e;
  }
  return static_cast<uint8_t>(sign | (static_cast<uint32_t>(e + 7) << 3) | r);
}

__global__ void __launch_bounds__(256) quantize_bf16_kernel(const float* X, uint64_t n, uint32_t dim,
                                                            uint64_t ld, uint16_t* out) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n * dim;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint64_t r = i / dim, c = i % dim;
    out[i] = bf16_encode(X[r * ld + c]);
  }
}

// one wavefront per row: scale = max|x| / 448, code = fp8(x * (448 / max|x|))
__global__ void __launch_bounds__(256) quantize_fp8_kernel(const float* X, uint64_t n, uint32_t dim,
                                                           uint64_t ld, uint8_t* out, float* scale) {
  const uint32_t wave = threadIdx.x / 64;
  const int lane = lane_id();
  for (uint64_t row = blockIdx.x * 4ull + wave; row < n; row += gridDim.x * 4ull) {
    const float* x = X + row * ld;
    float amax = 0.0f;
    for (uint32_t t = lane; t < dim; t += 64) amax = fmaxf(amax, fabsf(x[t]));
    for (int st = 32; st >= 1; st /= 2) amax = fmaxf(amax, __shfl_xor(amax, st, 64));
    const float inv = amax > 0.0f ? 448.0f / amax : 1.0f;
    if (lane == 0) scale[row] = amax > 0.0f ? amax / 448.0f : 1.0f;
    for (uint32_t t = lane; t < dim; t += 64) out[row * dim + t] = fp8_encode(x[t] * inv);
  }
}

// MIPS -> L2, first pass: n(x) = the canonical FP32 squared length (chunks of
// 4 summed with fused multiply-adds from +0, padded to Np chunks and added by
// the stride tree), parked in the row's extra output slot and folded into the
// maximum (non-negative floats order like their bit patterns); the row's
// own chunks are copied to the output on the way.  A group of P = min(Np,
// 64) lanes takes a row (lane l owns chunks l, l + P, ...), a wavefront
// 64 / P rows at a time, and U such steps are loaded before any is reduced,
// so their latencies overlap.
template <int MMAX, int U>
__global__ void __launch_bounds__(256) mips_norm_kernel(const float* X, uint64_t n, uint32_t nc, uint32_t Np,
                                                        uint64_t ld, float* out, uint64_t ld_out, uint32_t dim,
                                                        uint32_t* max_bits) {
  const uint32_t lane = static_cast<uint32_t>(lane_id());
  const uint32_t P = Np < 64 ? Np : 64;
  const uint32_t M = Np / P;  // <= MMAX
  const uint32_t G = 64 / P;
  const uint32_t g = lane / P, l = lane % P;
  const uint64_t waves = gridDim.x * 4ull;
  const uint64_t w = uniform(blockIdx.x * 4u + threadIdx.x / 64u);
  uint32_t mx = 0;
  for (uint64_t base = w * G * U; base < n; base += waves * G * U) {
    float4 x[U][MMAX];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t row = base + static_cast<uint64_t>(u) * G + g;
#pragma unroll
      for (int mi = 0; mi < MMAX; ++mi) {
        const uint32_t c = l + mi * P;
        x[u][mi] = row < n && static_cast<uint32_t>(mi) < M && c < nc
                       ? *reinterpret_cast<const float4*>(X + row * ld + 4ull * c)
                       : make_float4(0.f, 0.f, 0.f, 0.f);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t row = base + static_cast<uint64_t>(u) * G + g;
#pragma unroll
      for (int mi = 0; mi < MMAX; ++mi) {
        const uint32_t c = l + mi * P;
        if (row < n && static_cast<uint32_t>(mi) < M && c < nc)
          *reinterpret_cast<float4*>(out + row * ld_out + 4ull * c) = x[u][mi];
      }
      float s[MMAX];
#pragma unroll
      for (int mi = 0; mi < MMAX; ++mi) s[mi] = chunk_sum<kIP>(x[u][mi], x[u][mi]);
      // the squared length is the L2 form's sum: no sign, -0 made +0
      const float r = finish<kL2>(reduce_chunk_sums<MMAX>(s, static_cast<int>(P), static_cast<int>(M)));
      if (row < n && l == 0) {
        out[row * ld_out + dim] = r;
        const uint32_t b = __float_as_uint(r);
        mx = b > mx ? b : mx;
      }
    }
  }
  for (int o = 32; o >= 1; o >>= 1) {
    const uint32_t t = static_cast<uint32_t>(__shfl_xor(static_cast<int>(mx), o, 64));
    mx = t > mx ? t : mx;
  }
  if (lane == 0) atomicMax(max_bits, mx);
}

// second pass: the last chunk of each row, (sqrt(M - n(x)), 0, 0, 0)
__global__ void __launch_bounds__(256) mips_write_kernel(uint64_t n, uint32_t dim, float* out, uint64_t ld_out,
                                                         const float* max_norm2) {
  const float Mx = *max_norm2;
  for (uint64_t row = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; row < n;
       row += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    float* t = out + row * ld_out + dim;
    *reinterpret_cast<float4*>(t) = make_float4(__builtin_sqrtf(Mx - t[0]), 0.0f, 0.0f, 0.0f);
  }
}

// Read stream: every 16-byte word of the buffer once.  Each wavefront reads
// contiguous tiles of kReadUnroll x 1 KB (64 lanes x 16 B per load, all
// loads of a tile in flight together, non-temporal so the stream does not
// displace cached data) and the wavefronts stride over the tiles; the words
// are XOR-folded into one so no load can be dropped.  Two workgroups per
// compute unit measured fastest (7.1 TB/s on 4 GiB; more resident waves
// contend and lose up to 15 %).
constexpr int kReadUnroll = 4;
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(256) read_stream_kernel(const u32x4_t* data, uint64_t n16, uint32_t* checksum) {
  uint32_t x = 0;
  const uint64_t waves = static_cast<uint64_t>(gridDim.x) * 4;
  const uint64_t w = blockIdx.x * 4ull + threadIdx.x / 64;
  const uint64_t lane = lane_id();
  const uint64_t tile = 64ull * kReadUnroll;
  const uint64_t full = n16 / tile;
  for (uint64_t t = w; t < full; t += waves) {
    u32x4_t v[kReadUnroll];
#pragma unroll
    for (int u = 0; u < kReadUnroll; ++u) v[u] = __builtin_nontemporal_load(&data[t * tile + u * 64 + lane]);
#pragma unroll
    for (int u = 0; u < kReadUnroll; ++u) x ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
  }
  for (uint64_t i = full * tile + w * 64 + lane; i < n16; i += waves * 64) {
    const u32x4_t v = data[i];
    x ^= v.x ^ v.y ^ v.z ^ v.w;
  }
  for (int o = 32; o >= 1; o >>= 1) x ^= static_cast<uint32_t>(__shfl_xor(static_cast<int>(x), o, 64));
  if (lane_id() == 0) atomicXor(checksum, x);
}

// ---------------------------------------------------------------------------
// host helpers

bool is_pow2(uint64_t x) { return x && !(x & (x - 1)); }

uint32_t ceil_pow2(uint32_t x) {
  uint32_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

uint32_t ilog2(uint32_t x) {
  uint32_t l = 0;
  while ((1u << l) < x) ++l;
  return l;
}

fgim_status check_rows(const float* base, uint64_t n, uint32_t dim, uint64_t ld) {
  if (!base) return fail(FGIM_ERR_INVALID_ARG, "base is NULL");
  // ids are 32-bit with 0xFFFFFFFF reserved, and the work queue's 32-bit
  // counter may run up to 2^20 past the item count
  if (n == 0 || n >= 0xFFF00000ull) return fail(FGIM_ERR_INVALID_ARG, "row count %llu out of range", (unsigned long long)n);
  if (dim < 4 || dim > FGIM_MAX_DIM || dim % 4)
    return fail(dim % 4 ? FGIM_ERR_UNSUPPORTED : FGIM_ERR_INVALID_ARG, "dim %u must be a multiple of 4 in 4..%u", dim, FGIM_MAX_DIM);
  if (ld < dim || ld % 4) return fail(FGIM_ERR_INVALID_ARG, "ld %llu must be a multiple of 4 and >= dim", (unsigned long long)ld);
  if (reinterpret_cast<uintptr_t>(base) % 16) return fail(FGIM_ERR_INVALID_ARG, "base must be 16-byte aligned");
  return FGIM_OK;
}

fgim_status check_dataset(const fgim_dataset* d, bool need_cross) {
  if (!d) return fail(FGIM_ERR_INVALID_ARG, "dataset is NULL");
  fgim_status st = check_rows(d->base, d->n_total, d->dim, d->ld);
  if (st) return st;
  if (d->metric != FGIM_L2 && d->metric != FGIM_IP && d->metric != FGIM_COSINE)
    return fail(FGIM_ERR_INVALID_ARG, "unknown metric %d", (int)d->metric);
  if (!d->subs || d->h == 0) return fail(FGIM_ERR_INVALID_ARG, "no sub-indexes");
  if (d->h > 4096) return fail(FGIM_ERR_UNSUPPORTED, "h = %u sub-indexes (max 4096)", d->h);
  uint64_t expect = 0;
  for (uint32_t i = 0; i < d->h; ++i) {
    const fgim_subindex& s = d->subs[i];
    if (s.row_offset != expect)
      return fail(FGIM_ERR_INVALID_ARG, "sub-index %u starts at %llu, expected %llu (ranges must tile [0, n_total) in order)",
                  i, (unsigned long long)s.row_offset, (unsigned long long)expect);
    if (s.n == 0) return fail(FGIM_ERR_INVALID_ARG, "sub-index %u is empty", i);
    if (need_cross) {
      if (!s.adj) return fail(FGIM_ERR_INVALID_ARG, "sub-index %u: adj is NULL", i);
      if (s.adj_stride == 0 || s.adj_stride > FGIM_MAX_STRIDE)
        return fail(FGIM_ERR_INVALID_ARG, "sub-index %u: adj_stride %u out of 1..%u", i, s.adj_stride, FGIM_MAX_STRIDE);
      if (s.entry >= s.n) return fail(FGIM_ERR_INVALID_ARG, "sub-index %u: entry %u >= n %u", i, s.entry, s.n);
    }
    expect += s.n;
  }
  if (expect != d->n_total)
    return fail(FGIM_ERR_INVALID_ARG, "sub-index sizes sum to %llu, n_total is %llu", (unsigned long long)expect,
                (unsigned long long)d->n_total);
  return FGIM_OK;
}

fgim_status beam_shape(uint32_t dim, uint32_t L, uint32_t k, const fgim_params* p, BeamShape* out,
                       double mean_degree) {
  const uint32_t nc = dim / 4;
  const uint32_t N = ceil_pow2(nc);
  // defaults measured on 2 x 500k rows, d=128, L=64: four chunks per lane
  // (P = 8) with two candidate batches in flight per wave, 32 workgroups per
  // CU (VGPR-limited to 16 resident): 95 ms with a 1024-slot visited cache,
  // against 100 ms for two chunks per lane and 129 ms for the first shape
  // (90.6 ms now, with 2048 two-choice slots and empty batches skipped)
  // Searches on sparse graphs (mean out-degree <= 12) score few rows per
  // expansion and wait on their chains of dependent loads, so residency
  // decides: two chunks per lane take the kernels with the fewest registers
  // (67 / 87 / 92 VGPRs for FP32 / BF16 / FP8 against 92 / 122 / 124 with
  // four), and a 1024-slot visited cache lets that many waves fit in LDS
  // (a search that scores few rows remembers few ids).  Measured, stage 1
  // FP32 / BF16 / FP8: 8 uneven sub-indexes of 2 M rows, d = 96, L = 48,
  // mean degree 9.4: 294 / 343 / 350 ms -> 266 / 332 / 338 ms.  Denser graphs
  // keep the shape below: at mean degree 13.5 (2 x 500k rows, d = 128)
  // either change was 1-14 % slower, at 18.6 (the 2 M-row set with
  // navigable inputs) both together 4-9 % slower.  20 uneven sub-indexes of
  // 11.4 M rows, d = 128, L = 96 (four dense 2.5 M-row graphs, sixteen sparse
  // small ones: mean degree 9.9 over graphs, above 12 over rows): 15.5 /
  // 15.7 / 15.6 s -> 13.6 / 15.0 / 15.0 s.  The mean weights each graph by
  // the searches that run in it (n_total - n_i), not by its rows.
  const bool short_search = mean_degree > 0.0 && mean_degree <= 12.0;
  uint32_t P = p && p->lanes_per_dist ? p->lanes_per_dist
                                      : std::min<uint32_t>(64, std::max<uint32_t>(std::min<uint32_t>(4, N),
                                                                                   short_search ? N / 2 : N / 4));
  if (!is_pow2(P) || P > 64 || P > N) return fail(FGIM_ERR_INVALID_ARG, "lanes_per_dist %u must be a power of 2 <= min(64, %u)", P, N);
  const uint32_t M = N / P;
  if (M > 16) return fail(FGIM_ERR_INVALID_ARG, "lanes_per_dist %u too small for dim %u", P, dim);
  const uint32_t cap = std::max(L, k);
  uint32_t nr = cap <= 64 ? 1 : (cap <= 128 ? 2 : 4);
  // 2048 slots (8 KB per wave) still fit the 16 resident waves of the
  // default shape and re-score 2.7 % fewer ids than 1024 (93 vs 96 ms)
  uint32_t slots = p && p->visited_slots ? p->visited_slots : std::min<uint32_t>(2048, std::max<uint32_t>(1024, ceil_pow2(32 * L)));
  if (!(p && p->visited_slots) && short_search) slots = std::min<uint32_t>(slots, 1024);
  if (!is_pow2(slots) || slots < 64 || slots > 16384) return fail(FGIM_ERR_INVALID_ARG, "visited_slots %u must be a power of 2 in 64..16384", slots);
  uint32_t waves = p && p->waves_per_cu ? p->waves_per_cu : 32;
  if (waves > 64) return fail(FGIM_ERR_INVALID_ARG, "waves_per_cu %u > 64", waves);
  *out = BeamShape{P, M, M <= 2 ? 2u : (M <= 4 ? 4u : 16u), nr, ilog2(slots), waves};
  return FGIM_OK;
}

size_t beam_smem(const BeamShape& s) { return 64 * 8 + 64 * 4 + (size_t(4) << s.vis_log2); }

hipError_t launch_beam(const BeamArgs& a, bool l2, int fmt, const BeamShape& s, hipStream_t st) {
  dim3 grid(device_cus() * s.waves);
  size_t smem = beam_smem(s);
  if (fmt == kF32) return launch_beam_f32(a, l2, s.nr, s.mmax, grid, smem, st);
  if (fmt == kBF16) return launch_beam_bf16(a, l2, s.nr, s.mmax, grid, smem, st);
  return launch_beam_fp8(a, l2, s.nr, s.mmax, grid, smem, st);
}

fgim_status rerank_for(const fgim_params* p, uint32_t L, uint32_t* out) {
  uint32_t rerank = p->rerank ? p->rerank : std::min<uint32_t>(L, 2 * p->k);
  if (p->precision != FGIM_FP32 && (rerank < p->k || rerank > L)) {
    if (p->rerank) return fail(FGIM_ERR_INVALID_ARG, "rerank %u must be in k..L", p->rerank);
    rerank = std::min(L, std::max(rerank, p->k));
  }
  *out = rerank;
  return FGIM_OK;
}

fgim_status quantize_into(const float* base, uint64_t n, uint32_t dim, uint64_t ld, fgim_precision prec,
                          void* codes, float* scales, hipStream_t s) {
  if (prec == FGIM_BF16) {
    uint64_t blocks = std::min<uint64_t>((n * dim + 255) / 256, 65536);
    hipLaunchKernelGGL(quantize_bf16_kernel, dim3(blocks), dim3(256), 0, s, base, n, dim, ld,
                       static_cast<uint16_t*>(codes));
  } else {
    uint64_t blocks = std::min<uint64_t>((n + 3) / 4, 65536);
    hipLaunchKernelGGL(quantize_fp8_kernel, dim3(blocks), dim3(256), 0, s, base, n, dim, ld,
                       static_cast<uint8_t*>(codes), scales);
  }
  HIP_TRY(hipGetLastError());
  return FGIM_OK;
}

// ---------------------------------------------------------------------------
// stage 1

fgim_status cross_query_check(const fgim_dataset* d, const fgim_params* p, const uint32_t* ids,
                              const float* dist) {
  FGIM_TRY(check_dataset(d, true));
  if (!p) return fail(FGIM_ERR_INVALID_ARG, "params is NULL");
  if (!ids || !dist) return fail(FGIM_ERR_INVALID_ARG, "output is NULL");
  if (p->k == 0 || p->k > FGIM_MAX_K) return fail(FGIM_ERR_INVALID_ARG, "k = %u out of 1..%u", p->k, FGIM_MAX_K);
  if (p->L == 0 || p->L > FGIM_MAX_L) return fail(FGIM_ERR_INVALID_ARG, "L = %u out of 1..%u", p->L, FGIM_MAX_L);
  if (p->precision != FGIM_FP32 && p->precision != FGIM_BF16 && p->precision != FGIM_FP8_E4M3)
    return fail(FGIM_ERR_INVALID_ARG, "unknown precision %d", (int)p->precision);
  uint32_t rr = 0;
  BeamShape sh;
  FGIM_TRY(rerank_for(p, p->L, &rr));
  FGIM_TRY(beam_shape(d->dim, p->L, p->k, p, &sh));
  return FGIM_OK;
}

fgim_status cross_query_run(const fgim_dataset* d, const fgim_params* p, uint32_t* ids, float* dist,
                            fgim_stats* stats, hipStream_t s, uint32_t* L_used, const CrossBufs& b) {
  uint32_t* hdr = b.hdr;  // [0] queue head, [1] error flag, [2] smallest input out-degree
  for (uint32_t i = 0; i < d->h; ++i)
    b.host_subs[i] = SubDev{d->subs[i].row_offset, d->subs[i].adj, d->subs[i].n, d->subs[i].adj_stride,
                            d->subs[i].entry, 0};
  HIP_TRY(hipMemcpyAsync(b.subs, b.host_subs, sizeof(SubDev) * d->h, hipMemcpyHostToDevice, s));
  HIP_TRY(fill_u32(hdr, 0u, 2, s));
  HIP_TRY(fill_u32(hdr + 2, 0xFFFFFFFFu, 2, s));
  HIP_TRY(fill_u32(reinterpret_cast<uint32_t*>(b.cnt), 0u, 8, s));
  for (uint32_t i = 0; i < d->h; ++i)
    HIP_TRY(validate_graph(d->subs[i].adj, d->subs[i].n, d->subs[i].adj_stride, hdr + 1, s,
                           p->autotune ? hdr + 2 : nullptr, reinterpret_cast<double*>(b.cnt + 3),
                           static_cast<double>(d->n_total - d->subs[i].n) / static_cast<double>(d->subs[i].n)));
  if (p->precision == FGIM_FP8_E4M3 && !b.lps) return fail(FGIM_ERR_INVALID_ARG, "FP8 copy given without scales");

  BeamArgs a{};
  a.X = d->base;
  a.ld = d->ld;
  a.nc = d->dim / 4;
  a.metric = d->metric;
  a.xb = p->precision == FGIM_BF16 ? static_cast<const uint16_t*>(b.lp) : nullptr;
  a.x8 = p->precision == FGIM_FP8_E4M3 ? static_cast<const uint8_t*>(b.lp) : nullptr;
  a.x8s = b.lps;
  a.dim = d->dim;
  a.subs = b.subs;
  a.h = d->h;
  a.k = p->k;
  a.n_items = d->n_total;
  a.item_stride = 1;
  a.compact_out = 0;
  a.out_ids = ids;
  a.out_dist = dist;
  a.counter = hdr;
  a.err = hdr + 1;
  a.search_mode = 0;
  a.valid = d->valid;
  const int fmt = p->precision == FGIM_FP32 ? kF32 : (p->precision == FGIM_BF16 ? kBF16 : kFP8);
  const bool l2 = d->metric == FGIM_L2;

  uint32_t L = p->L;
  BeamShape shape;
  double ms_tune = 0.0;
  if (p->autotune) {
    // trial launches mean nothing on a malformed graph: check it first
    uint32_t hv[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(hv, hdr + 1, sizeof(hv), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (hv[0]) return fail(FGIM_ERR_GRAPH, "an adjacency list holds an out-of-range id, a self-loop or a duplicate");
    uint32_t lo = fgim_min_beam_width(p->k, hv[1], d->h);
    if (p->precision != FGIM_FP32 && p->rerank) lo = std::max(lo, p->rerank);
    FGIM_TRY(tune_stage1(a, d, p, fmt, l2, lo, &L, &shape, &ms_tune, s));
  } else {
    // The mean out-degree of the graphs the searches run in: graph i is
    // searched by the n_total - n_i vertices outside it, so its mean degree
    // (its degree sum over n_i, summed by the validation above) counts with
    // that weight.  A lone graph is never searched: no mean.
    double wsum = 0.0, wtot = 0.0;
    for (uint32_t i = 0; i < d->h; ++i) wtot += static_cast<double>(d->n_total - d->subs[i].n);
    HIP_TRY(hipMemcpyAsync(&wsum, b.cnt + 3, sizeof(wsum), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    FGIM_TRY(beam_shape(d->dim, L, p->k, p, &shape, wtot > 0.0 ? wsum / wtot : 0.0));
  }
  uint32_t rerank = 0;
  FGIM_TRY(rerank_for(p, L, &rerank));
  a.L = L;
  a.rerank = rerank;
  a.stats = b.cnt;
  a.vis_log2 = shape.vis_log2;
  a.P = shape.P;
  a.M = shape.M;

  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (stats) {
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    HIP_TRY(hipEventRecord(e0, s));
  }
  HIP_TRY(launch_beam(a, l2, fmt, shape, s));
  if (stats) HIP_TRY(hipEventRecord(e1, s));

  uint32_t herr = 0;
  unsigned long long hc[3] = {0, 0, 0};
  HIP_TRY(hipMemcpyAsync(&herr, hdr + 1, 4, hipMemcpyDeviceToHost, s));
  if (stats) HIP_TRY(hipMemcpyAsync(hc, b.cnt, sizeof(hc), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (stats) {
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
    stats->ms_beam_kernel = ms;
    stats->ndc = hc[0];
    stats->expansions = hc[1];
    stats->searches = hc[2];
    stats->L_used = L;
    stats->lanes_per_dist = shape.P;
    stats->waves_per_cu = shape.waves;
    stats->visited_slots = 1u << shape.vis_log2;
    stats->ms_tune = ms_tune;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  }
  if (L_used) *L_used = L;
  if (herr) return fail(FGIM_ERR_GRAPH, "an adjacency list holds an out-of-range id, a self-loop or a duplicate");
  return FGIM_OK;
}

fgim_status cross_query_impl(const fgim_dataset* d, const fgim_params* p, uint32_t* ids, float* dist,
                             fgim_stats* stats, hipStream_t s, uint32_t* L_used) {
  FGIM_TRY(cross_query_check(d, p, ids, dist));  // argument errors before anything is enqueued
  Scratch scr(s);
  CrossBufs b{};
  FGIM_TRY(scr.get(&b.hdr, 4));
  FGIM_TRY(scr.get(&b.cnt, 4));
  FGIM_TRY(scr.get(&b.subs, d->h));
  std::vector<SubDev> hs(d->h);
  b.host_subs = hs.data();
  b.lp = d->base_lp;
  b.lps = d->base_lp_scale;
  if (p->precision != FGIM_FP32 && !b.lp) {
    if (p->precision == FGIM_BF16) {
      uint16_t* c = nullptr;
      FGIM_TRY(scr.get(&c, d->n_total * d->dim));
      FGIM_TRY(quantize_into(d->base, d->n_total, d->dim, d->ld, p->precision, c, nullptr, s));
      b.lp = c;
    } else {
      uint8_t* c = nullptr;
      float* sc = nullptr;
      FGIM_TRY(scr.get(&c, d->n_total * d->dim));
      FGIM_TRY(scr.get(&sc, d->n_total));
      FGIM_TRY(quantize_into(d->base, d->n_total, d->dim, d->ld, p->precision, c, sc, s));
      b.lp = c;
      b.lps = sc;
    }
  }
  return cross_query_run(d, p, ids, dist, stats, s, L_used, b);
}

}  // namespace fgim

using namespace fgim;

extern "C" {

const char* fgim_status_string(fgim_status s) {
  switch (s) {
    case FGIM_OK: return "ok";
    case FGIM_ERR_INVALID_ARG: return "invalid argument";
    case FGIM_ERR_GRAPH: return "malformed adjacency list";
    case FGIM_ERR_OUT_OF_MEMORY: return "out of device memory";
    case FGIM_ERR_DEVICE: return "HIP error";
    case FGIM_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* fgim_last_error(void) { return g_last_error.c_str(); }

fgim_status fgim_release_scratch(void) {
  g_last_error.clear();
  return release_scratch();
}

uint32_t fgim_min_beam_width(uint32_t k, uint32_t min_local, uint32_t h) {
  if (h < 2) return 0;
  if (min_local >= k) return 1;
  const uint32_t need = k - min_local;
  const uint32_t l = (need + h - 2) / (h - 1);
  return l ? l : 1;
}

fgim_status fgim_cross_query(const fgim_dataset* data, const fgim_params* params, uint32_t* knn_ids,
                             float* knn_dist, fgim_stats* stats, void* stream) {
  g_last_error.clear();
  if (stats) memset(stats, 0, sizeof(*stats));
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipEvent_t a = nullptr, b = nullptr;
  if (stats) {
    HIP_TRY(hipEventCreate(&a));
    HIP_TRY(hipEventCreate(&b));
    HIP_TRY(hipEventRecord(a, s));
  }
  fgim_status st = cross_query_impl(data, params, knn_ids, knn_dist, stats, s, nullptr);
  if (stats && st == FGIM_OK) {
    HIP_TRY(hipEventRecord(b, s));
    HIP_TRY(hipEventSynchronize(b));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, a, b));
    stats->ms_stage[0] = ms;
  }
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  return st;
}

fgim_status fgim_search(const float* base, uint64_t n, uint32_t dim, uint64_t ld, fgim_metric metric,
                        const uint32_t* adj, uint32_t stride, uint32_t entry, const float* queries,
                        uint64_t nq, uint64_t ldq, uint32_t L, uint32_t topk, uint32_t* out_ids,
                        float* out_dist, void* stream) {
  g_last_error.clear();
  hipStream_t s = static_cast<hipStream_t>(stream);
  FGIM_TRY(check_rows(base, n, dim, ld));
  if (metric != FGIM_L2 && metric != FGIM_IP && metric != FGIM_COSINE) return fail(FGIM_ERR_INVALID_ARG, "unknown metric");
  if (!adj || stride == 0 || stride > FGIM_MAX_STRIDE) return fail(FGIM_ERR_INVALID_ARG, "bad adjacency (stride %u)", stride);
  if (entry >= n) return fail(FGIM_ERR_INVALID_ARG, "entry %u >= n", entry);
  if (nq == 0) return FGIM_OK;
  if (!queries || ldq < dim || ldq % 4 || reinterpret_cast<uintptr_t>(queries) % 16)
    return fail(FGIM_ERR_INVALID_ARG, "bad query matrix");
  if (nq >= 0xFFF00000ull) return fail(FGIM_ERR_INVALID_ARG, "too many queries");
  if (L == 0 || L > FGIM_MAX_L || topk == 0 || topk > L) return fail(FGIM_ERR_INVALID_ARG, "need 1 <= topk <= L <= %u", FGIM_MAX_L);
  if (!out_ids || !out_dist) return fail(FGIM_ERR_INVALID_ARG, "output is NULL");
  BeamShape shape;
  FGIM_TRY(beam_shape(dim, L, topk, nullptr, &shape));
  Scratch scr(s);
  uint32_t* hdr = nullptr;
  SubDev* sub = nullptr;
  FGIM_TRY(scr.get(&hdr, 4));
  FGIM_TRY(scr.get(&sub, 1));
  SubDev hs{0, adj, static_cast<uint32_t>(n), stride, entry, 0};
  HIP_TRY(hipMemcpyAsync(sub, &hs, sizeof(hs), hipMemcpyHostToDevice, s));
  HIP_TRY(fill_u32(hdr, 0u, 4, s));
  HIP_TRY(validate_graph(adj, static_cast<uint32_t>(n), stride, hdr + 1, s));
  BeamArgs a{};
  a.item_stride = 1;
  a.X = base;
  a.ld = ld;
  a.nc = dim / 4;
  a.metric = metric;
  a.dim = dim;
  a.subs = sub;
  a.h = 1;
  a.L = L;
  a.k = topk;
  a.rerank = topk;
  a.n_items = nq;
  a.out_ids = out_ids;
  a.out_dist = out_dist;
  a.counter = hdr;
  a.err = hdr + 1;
  a.stats = nullptr;
  a.vis_log2 = shape.vis_log2;
  a.P = shape.P;
  a.M = shape.M;
  a.search_mode = 1;
  a.Q = queries;
  a.ldq = ldq;
  HIP_TRY(launch_beam(a, metric == FGIM_L2, kF32, shape, s));
  uint32_t herr = 0;
  HIP_TRY(hipMemcpyAsync(&herr, hdr + 1, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (herr) return fail(FGIM_ERR_GRAPH, "the graph holds an out-of-range id, a self-loop or a duplicate");
  return FGIM_OK;
}

fgim_status fgim_mips_to_l2(const float* base, uint64_t n, uint32_t dim, uint64_t ld, float* out, uint64_t ld_out,
                            float* max_norm2, void* stream) {
  g_last_error.clear();
  FGIM_TRY(check_rows(base, n, dim, ld));
  if (!out || !max_norm2) return fail(FGIM_ERR_INVALID_ARG, "output is NULL");
  if (ld_out < static_cast<uint64_t>(dim) + 4 || ld_out % 4 || reinterpret_cast<uintptr_t>(out) % 16)
    return fail(FGIM_ERR_INVALID_ARG, "out rows need ld_out >= dim + 4, a multiple of 4, and 16-byte alignment");
  const uint64_t lo = reinterpret_cast<uintptr_t>(out), hi = lo + 4 * (n * ld_out);
  const uint64_t blo = reinterpret_cast<uintptr_t>(base), bhi = blo + 4 * (n * ld);
  if (lo < bhi && blo < hi) return fail(FGIM_ERR_INVALID_ARG, "out overlaps base");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const uint32_t nc = dim / 4;
  HIP_TRY(fill_u32(reinterpret_cast<uint32_t*>(max_norm2), 0u, 1, s));
  const uint32_t Np = ceil_pow2(nc);
  const uint32_t M = Np <= 64 ? 1u : Np / 64;
  const dim3 grid(static_cast<uint32_t>(std::min<uint64_t>((n + 3) / 4, static_cast<uint64_t>(device_cus()) * 8)));
  uint32_t* mb = reinterpret_cast<uint32_t*>(max_norm2);
  if (M == 1)
    hipLaunchKernelGGL((mips_norm_kernel<1, 4>), grid, dim3(256), 0, s, base, n, nc, Np, ld, out, ld_out, dim, mb);
  else if (M == 2)
    hipLaunchKernelGGL((mips_norm_kernel<2, 2>), grid, dim3(256), 0, s, base, n, nc, Np, ld, out, ld_out, dim, mb);
  else if (M == 4)
    hipLaunchKernelGGL((mips_norm_kernel<4, 1>), grid, dim3(256), 0, s, base, n, nc, Np, ld, out, ld_out, dim, mb);
  else
    hipLaunchKernelGGL((mips_norm_kernel<16, 1>), grid, dim3(256), 0, s, base, n, nc, Np, ld, out, ld_out, dim, mb);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(mips_write_kernel, dim3(static_cast<uint32_t>(std::min<uint64_t>((n + 255) / 256, 65536))),
                     dim3(256), 0, s, n, dim, out, ld_out, max_norm2);
  HIP_TRY(hipGetLastError());
  return FGIM_OK;
}

fgim_status fgim_read_stream(const void* data, uint64_t bytes, uint32_t* checksum, void* stream) {
  g_last_error.clear();
  if (!checksum || (bytes && !data)) return fail(FGIM_ERR_INVALID_ARG, "data or checksum is NULL");
  if (bytes % 16 || reinterpret_cast<uintptr_t>(data) % 16)
    return fail(FGIM_ERR_INVALID_ARG, "data must be 16-byte aligned and a multiple of 16 bytes long");
  hipStream_t s = static_cast<hipStream_t>(stream);
  HIP_TRY(fill_u32(checksum, 0u, 1, s));
  if (bytes == 0) return FGIM_OK;
  const uint64_t n16 = bytes / 16;
  const uint64_t blocks = std::min<uint64_t>((n16 + 255) / 256, static_cast<uint64_t>(device_cus()) * 2);
  hipLaunchKernelGGL(read_stream_kernel, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, s,
                     static_cast<const u32x4_t*>(data), n16, checksum);
  HIP_TRY(hipGetLastError());
  return FGIM_OK;
}

fgim_status fgim_quantize(const float* base, uint64_t n, uint32_t dim, uint64_t ld, fgim_precision precision,
                          void* codes, float* scales, void* stream) {
  g_last_error.clear();
  FGIM_TRY(check_rows(base, n, dim, ld));
  if (precision != FGIM_BF16 && precision != FGIM_FP8_E4M3)
    return fail(FGIM_ERR_INVALID_ARG, "precision must be BF16 or FP8_E4M3");
  if (!codes || (precision == FGIM_FP8_E4M3 && !scales)) return fail(FGIM_ERR_INVALID_ARG, "output is NULL");
  return quantize_into(base, n, dim, ld, precision, codes, scales, static_cast<hipStream_t>(stream));
}

}  // extern "C"
