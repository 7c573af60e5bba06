// Stage 2 of FGIM: k-NNG refinement (Section 4.2, Algorithm 3) in
// synchronous rounds, with indegree repair (Algorithm 4) after every round.
//
// Lists are held as sorted uint64 keys (delta, id) plus a flag word per slot
// (bit 0 new, bit 1 replaced); the indegrees T and the counts of new
// in-edges are kept current by apply and repair.  One round is a fixed
// sequence of kernels with no host round trip: the first round runs
// directly while the host captures one round into a hipGraph, and the other
// rounds replay it.  The screened-pair and proposal buffers are sized from
// the demand seen in earlier calls; a round that needs more is detected at
// the end (64-bit demand counters) and the rounds run again with larger
// buffers.
//   Visit   active vertices from the maintained counts; reverse lists of
//           new and old entries as a CSR (segment 2v: u with v new in u's
//           list, 2v+1: old), grouped without global atomics
//           (group_records)
//   Update  Cn(u) = fwd_new U rev_new and Co(u) = (fwd_old U rev_old) \ Cn,
//           reverse lists cut to their k_rev best by (delta, u); every
//           cross-sub-index pair of Cn^2 U Cn x Co proposes each end to the
//           other when it beats that end's current worst entry.  When
//           |Cn| + |Co| <= 128: cand_kernel builds the sets, join_mfma_kernel
//           screens the pairs on MFMA with a rigorous error bound and
//           recheck_kernel scores the survivors in canonical FP32 (a vertex
//           without a new candidate has no pair and stages no row); otherwise
//           join_kernel scores every pair in FP32 from rows staged in LDS.
//           Proposals are appended to a global buffer and grouped by target
//           (group_records).
//   apply   per target: first k of the snapshot list (entries turn old) and
//           its proposals (entries new), one entry per id.
//   repair  ordered list of zero-indegree vertices, then Algorithm 4 in one
//           workgroup in order-exact speculative batches (two steps per
//           wavefront slot for k <= 32).
// Every step's result is independent of scheduling: CSR segments are
// consumed through order-independent top-k selections under the total
// order of keys, so the output is bit-identical to the sequential oracle.
#include <string.h>

#include <mutex>

#include "fgim_internal.h"
#include "graph_util.h"
#include "mfma_util.h"
#include "host_util.h"

namespace fgim {

// ---------------------------------------------------------------------------
// exclusive scan (three passes, 1024 elements per block)

constexpr uint32_t kScanBlock = 1024;

__global__ void __launch_bounds__(256) scan_sums_kernel(const uint32_t* in, uint64_t n, uint32_t* sums) {
  __shared__ uint32_t red[256];
  const uint64_t base = blockIdx.x * static_cast<uint64_t>(kScanBlock);
  uint32_t s = 0;
  for (uint32_t i = threadIdx.x; i < kScanBlock; i += 256) {
    const uint64_t j = base + i;
    if (j < n) s += in[j];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = red[0];
}

// exclusive scan of the nb block sums in place; sums[nb] = total
__global__ void __launch_bounds__(1024) scan_top_kernel(uint32_t* sums, uint64_t nb) {
  __shared__ uint32_t buf[1024];
  uint32_t carry = 0;
  for (uint64_t base = 0; base < nb; base += 1024) {
    const uint64_t j = base + threadIdx.x;
    const uint32_t v = j < nb ? sums[j] : 0u;
    buf[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      const uint32_t t = threadIdx.x >= static_cast<uint32_t>(off) ? buf[threadIdx.x - off] : 0u;
      __syncthreads();
      buf[threadIdx.x] += t;
      __syncthreads();
    }
    if (j < nb) sums[j] = carry + buf[threadIdx.x] - v;
    const uint32_t tot = buf[1023];
    __syncthreads();
    carry += tot;
  }
  if (threadIdx.x == 0) sums[nb] = carry;
}

__global__ void __launch_bounds__(256) scan_apply_kernel(const uint32_t* in, uint64_t n, const uint32_t* sums,
                                                         uint64_t nb, uint32_t* out) {
  __shared__ uint32_t tsum[256];
  const uint64_t base = blockIdx.x * static_cast<uint64_t>(kScanBlock) + threadIdx.x * 4ull;
  uint32_t v[4], run = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    v[i] = base + i < n ? in[base + i] : 0u;
    run += v[i];
  }
  tsum[threadIdx.x] = run;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const uint32_t t = threadIdx.x >= static_cast<uint32_t>(off) ? tsum[threadIdx.x - off] : 0u;
    __syncthreads();
    tsum[threadIdx.x] += t;
    __syncthreads();
  }
  uint32_t acc = sums[blockIdx.x] + tsum[threadIdx.x] - run;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    if (base + i < n) out[base + i] = acc;
    acc += v[i];
  }
  if (blockIdx.x == nb - 1 && threadIdx.x == 0) out[n] = sums[nb];
}

uint64_t scan_tmp_words(uint64_t n) { return (n + kScanBlock - 1) / kScanBlock + 1; }

hipError_t exclusive_scan(const uint32_t* in, uint32_t* out, uint64_t n, uint32_t* tmp, hipStream_t s) {
  const uint64_t nb = (n + kScanBlock - 1) / kScanBlock;
  if (nb == 0) return fill_u32(out, 0u, 1, s);
  hipLaunchKernelGGL(scan_sums_kernel, dim3(static_cast<uint32_t>(nb)), dim3(256), 0, s, in, n, tmp);
  hipLaunchKernelGGL(scan_top_kernel, dim3(1), dim3(1024), 0, s, tmp, nb);
  hipLaunchKernelGGL(scan_apply_kernel, dim3(static_cast<uint32_t>(nb)), dim3(256), 0, s, in, n, tmp, nb, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Records (segment, value) grouped by segment into a CSR, with atomics in
// LDS only.  A move pass: each of G workgroups takes one contiguous share
// of the records and counts its records per bucket of 2^shift consecutive
// segments (the counts form a bucket-major matrix); an exclusive scan of the
// matrix gives every (bucket, workgroup) pair its run of the output, the
// runs of one bucket contiguous; each workgroup moves its records into its
// runs.  Two move passes run: the first into at most 64 coarse buckets, the
// second, over the first's output, into up to 4096 fine buckets.  A
// workgroup's stores thus go to a few dozen runs at a time, long enough for
// L2 to complete their lines (a single pass into 2048 buckets left 4-8 byte
// stores in about 2000 runs per workgroup and wrote about five times the
// records' bytes).  Last, one workgroup per fine bucket counts its records
// per segment, scans the counts, writes the segments' offsets and places
// every record in its segment.  The order of the records within a segment
// is not fixed; every reader of these segments selects from them under the
// total order of keys.

constexpr uint32_t kBucketMax = 4096;     // fine buckets
constexpr uint32_t kCoarseBits = 6;       // coarse bucket = 64 fine buckets
constexpr uint32_t kBucketWindow = 4096;  // segments a placing workgroup counts at a time
constexpr uint32_t kBucketThreads = 512;
constexpr int kBucketUnroll = 4;          // records per thread in flight

struct BucketPlan {
  uint64_t nseg;
  uint32_t shift1, C1;  // coarse bucket of segment s: s >> shift1
  uint32_t shift2, C2;  // fine bucket: s >> shift2
  uint32_t G, G2;       // workgroups of the coarse and the fine count / move passes
  uint64_t words1() const { return static_cast<uint64_t>(C1) * G; }
  uint64_t words2() const { return static_cast<uint64_t>(C2) * G2; }
};

// workgroups of the fine pass per CU: its count matrix has C2 x G2 words,
// each workgroup's column written and read at a stride of G2 words; one per
// CU measured 1.2 ms (2 %) faster over a refinement of 2 x 500k rows than
// four, two in between
constexpr uint32_t kFineGroupsPerCu = 1;

BucketPlan bucket_plan(uint64_t nseg, uint64_t max_records) {
  BucketPlan p{};
  p.nseg = nseg;
  auto buckets = [nseg](uint32_t sh) {
    return static_cast<uint32_t>(std::max<uint64_t>((nseg + (1ull << sh) - 1) >> sh, 1));
  };
  while (buckets(p.shift2) > kBucketMax) ++p.shift2;
  p.shift1 = p.shift2 + kCoarseBits;
  p.C1 = buckets(p.shift1);
  p.C2 = buckets(p.shift2);
  const uint64_t g = (max_records + 16383) / 16384;
  p.G = static_cast<uint32_t>(std::min<uint64_t>(std::max<uint64_t>(g, 1), 4ull * device_cus()));
  p.G2 = static_cast<uint32_t>(std::min<uint64_t>(std::max<uint64_t>(g, 1), uint64_t(kFineGroupsPerCu) * device_cus()));
  return p;
}

// proposals: record i = (target ptgt[i], key pkey[i]) for i < min(*total, cap)
struct PropRecords {
  const uint32_t* tgt;
  const uint64_t* key;
  const uint32_t* total;
  uint32_t cap;
  FGIM_DEV uint64_t count() const { return min(*total, cap); }
  FGIM_DEV bool seg_of(uint64_t i, uint32_t& seg) const {
    seg = tgt[i];
    return true;
  }
  FGIM_DEV uint64_t value(uint64_t i) const { return key[i]; }
};

// records of a first move pass: record i = (seg[i], val[i]) for i < *total
struct MovedRecords {
  const uint32_t* seg;
  const uint64_t* val;
  const uint32_t* total;
  FGIM_DEV uint64_t count() const { return *total; }
  FGIM_DEV bool seg_of(uint64_t i, uint32_t& s) const {
    s = seg[i];
    return true;
  }
  FGIM_DEV uint64_t value(uint64_t i) const { return val[i]; }
};

// reverse entries of a synchronous Visit: list entry i, u -> t with u = i / k,
// gives the record (2t if the entry is new, else 2t + 1; key (stored delta,
// u)).  Old entries of an inactive target give none: no join reads them.
// active: one bit per vertex (bit t & 31 of word t >> 5), small enough to
// stay in L2 for the random lookups.
struct RevRecords {
  const uint64_t* keys;
  const uint32_t* flags;
  const uint32_t* active;
  uint64_t nk;
  uint32_t k;
  FGIM_DEV uint64_t count() const { return nk; }
  FGIM_DEV bool seg_of(uint64_t i, uint32_t& seg) const {
    const uint64_t kk = keys[i];
    if (kk == kSentinel) return false;
    const uint32_t t = key_id(kk);
    const bool isnew = flags[i] & kFlagNew;
    if (!isnew && !((active[t >> 5] >> (t & 31u)) & 1u)) return false;
    seg = 2u * t + (isnew ? 0u : 1u);
    return true;
  }
  FGIM_DEV uint64_t value(uint64_t i) const {
    return (keys[i] & 0xFFFFFFFF00000000ull) | (static_cast<uint32_t>(i) / k);  // nk < 2^32
  }
};

// pass (1): mat[b G + g] = records of workgroup g's share in bucket b
template <class Src>
__global__ void __launch_bounds__(kBucketThreads) bucket_count_kernel(Src src, uint32_t shift, uint32_t C,
                                                                      uint32_t* mat) {
  __shared__ uint32_t hist[kBucketMax];
  for (uint32_t b = threadIdx.x; b < C; b += kBucketThreads) hist[b] = 0u;
  __syncthreads();
  const uint64_t n = src.count(), G = gridDim.x;
  const uint64_t lo = n * blockIdx.x / G, hi = n * (blockIdx.x + 1) / G;
  for (uint64_t i0 = lo + threadIdx.x; i0 < hi; i0 += kBucketUnroll * kBucketThreads) {
    uint32_t seg[kBucketUnroll];
    bool ok[kBucketUnroll];
#pragma unroll
    for (int u = 0; u < kBucketUnroll; ++u) {
      const uint64_t i = i0 + static_cast<uint64_t>(u) * kBucketThreads;
      ok[u] = i < hi && src.seg_of(i, seg[u]);
    }
#pragma unroll
    for (int u = 0; u < kBucketUnroll; ++u)
      if (ok[u]) atomicAdd(&hist[seg[u] >> shift], 1u);
  }
  __syncthreads();
  for (uint32_t b = threadIdx.x; b < C; b += kBucketThreads) mat[static_cast<uint64_t>(b) * G + blockIdx.x] = hist[b];
}

// pass (3): the share's records into their runs (moff: the scanned matrix)
template <class Src>
__global__ void __launch_bounds__(kBucketThreads) bucket_move_kernel(Src src, uint32_t shift, uint32_t C,
                                                                     const uint32_t* moff, uint32_t* cseg,
                                                                     uint64_t* cval) {
  __shared__ uint32_t cur[kBucketMax];
  const uint64_t n = src.count(), G = gridDim.x;
  for (uint32_t b = threadIdx.x; b < C; b += kBucketThreads) cur[b] = moff[static_cast<uint64_t>(b) * G + blockIdx.x];
  __syncthreads();
  const uint64_t lo = n * blockIdx.x / G, hi = n * (blockIdx.x + 1) / G;
  for (uint64_t i0 = lo + threadIdx.x; i0 < hi; i0 += kBucketUnroll * kBucketThreads) {
    uint32_t seg[kBucketUnroll];
    bool ok[kBucketUnroll];
    uint64_t val[kBucketUnroll];
#pragma unroll
    for (int u = 0; u < kBucketUnroll; ++u) {
      const uint64_t i = i0 + static_cast<uint64_t>(u) * kBucketThreads;
      ok[u] = i < hi && src.seg_of(i, seg[u]);
      val[u] = ok[u] ? src.value(i) : 0ull;
    }
#pragma unroll
    for (int u = 0; u < kBucketUnroll; ++u) {
      if (!ok[u]) continue;
      const uint32_t pos = atomicAdd(&cur[seg[u] >> shift], 1u);
      cseg[pos] = seg[u];
      cval[pos] = val[u];
    }
  }
}

// pass (4): bucket b's records lie in [moff[b G], moff[(b + 1) G]) (the
// scan's total closes the last bucket); they are counted per segment a
// window of segments at a time, and placed.  off[nseg] = the total.
__global__ void __launch_bounds__(kBucketThreads) bucket_place_kernel(const uint32_t* moff, uint32_t G, uint32_t shift,
                                                                      uint32_t C, uint64_t nseg, const uint32_t* cseg,
                                                                      const uint64_t* cval, uint32_t* off,
                                                                      uint64_t* out) {
  __shared__ uint32_t cnt[kBucketWindow];
  __shared__ uint32_t wsum[kBucketThreads / 64];
  const uint32_t b = blockIdx.x;
  const uint32_t r0 = uniform(moff[static_cast<uint64_t>(b) * G]);
  const uint32_t r1 = uniform(moff[static_cast<uint64_t>(b + 1) * G]);
  const uint64_t s0 = static_cast<uint64_t>(b) << shift;
  const uint64_t s_end = static_cast<uint64_t>(b + 1) << shift;
  const uint64_t s1 = s_end < nseg ? s_end : nseg;
  const uint32_t wid = threadIdx.x / 64, lane = lane_id();
  uint32_t base = r0;
  for (uint64_t w0 = s0; w0 < s1; w0 += kBucketWindow) {
    const uint32_t wn = static_cast<uint32_t>(s1 - w0 < kBucketWindow ? s1 - w0 : kBucketWindow);
    for (uint32_t i = threadIdx.x; i < wn; i += kBucketThreads) cnt[i] = 0u;
    __syncthreads();
    for (uint32_t r = r0 + threadIdx.x; r < r1; r += kBucketThreads) {
      const uint64_t sg = cseg[r];
      if (sg >= w0 && sg < w0 + wn) atomicAdd(&cnt[sg - w0], 1u);
    }
    __syncthreads();
    // exclusive scan of the window's counts, kBucketThreads at a time
    uint32_t carry = base;
    for (uint32_t c0 = 0; c0 < wn; c0 += kBucketThreads) {
      const uint32_t i = c0 + threadIdx.x;
      const uint32_t v = i < wn ? cnt[i] : 0u;
      uint32_t x = v;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, 64);
        if (lane >= static_cast<uint32_t>(d)) x += y;
      }
      if (lane == 63) wsum[wid] = x;
      __syncthreads();
      uint32_t before = carry, total = 0;
#pragma unroll
      for (uint32_t w = 0; w < kBucketThreads / 64; ++w) {
        before += w < wid ? wsum[w] : 0u;
        total += wsum[w];
      }
      if (i < wn) {
        cnt[i] = before + x - v;
        off[w0 + i] = before + x - v;
      }
      carry += total;
      __syncthreads();
    }
    for (uint32_t r = r0 + threadIdx.x; r < r1; r += kBucketThreads) {
      const uint64_t sg = cseg[r];
      if (sg >= w0 && sg < w0 + wn) out[atomicAdd(&cnt[sg - w0], 1u)] = cval[r];
    }
    __syncthreads();
    base = carry;
  }
  if (b == C - 1 && threadIdx.x == 0) off[nseg] = r1;
}

// the CSR (off: nseg + 1, out) of the records of src.  mat / moff hold
// plan.words2() and plan.words2() + 1 words (the coarse pass uses their
// head, of words1() + 1, and its total stays there for the fine pass);
// (seg1, val1) and (seg2, val2) hold one slot per record.
template <class Src>
hipError_t group_records(const Src& src, const BucketPlan& plan, uint32_t* mat, uint32_t* moff, uint32_t* mat2,
                         uint32_t* moff2, uint32_t* scan_tmp, uint32_t* seg1, uint64_t* val1, uint32_t* seg2,
                         uint64_t* val2, uint32_t* off, uint64_t* out, hipStream_t s) {
  hipError_t e;
  hipLaunchKernelGGL(bucket_count_kernel<Src>, dim3(plan.G), dim3(kBucketThreads), 0, s, src, plan.shift1, plan.C1,
                     mat);
  if ((e = exclusive_scan(mat, moff, plan.words1(), scan_tmp, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(bucket_move_kernel<Src>, dim3(plan.G), dim3(kBucketThreads), 0, s, src, plan.shift1, plan.C1,
                     moff, seg1, val1);
  const MovedRecords mid{seg1, val1, moff + plan.words1()};
  hipLaunchKernelGGL(bucket_count_kernel<MovedRecords>, dim3(plan.G2), dim3(kBucketThreads), 0, s, mid, plan.shift2,
                     plan.C2, mat2);
  if ((e = exclusive_scan(mat2, moff2, plan.words2(), scan_tmp, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(bucket_move_kernel<MovedRecords>, dim3(plan.G2), dim3(kBucketThreads), 0, s, mid, plan.shift2,
                     plan.C2, moff2, seg2, val2);
  hipLaunchKernelGGL(bucket_place_kernel, dim3(plan.C2), dim3(kBucketThreads), 0, s, moff2, plan.G2, plan.shift2,
                     plan.C2, plan.nseg, seg2, val2, off, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// list conversion

__global__ void to_keys_kernel(const uint32_t* ids, const float* dist, uint64_t nk, uint64_t* keys,
                               uint32_t* flags) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < nk;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint32_t v = ids[i];
    keys[i] = v == kNone ? kSentinel : make_key(dist[i] + 0.0f, v);
    flags[i] = v == kNone ? 0u : kFlagNew;
  }
}

__global__ void from_keys_kernel(const uint64_t* keys, uint64_t nk, uint32_t* ids, float* dist) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < nk;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint64_t k = keys[i];
    ids[i] = k == kSentinel ? kNone : key_id(k);
    dist[i] = key_dist(k);
  }
}

__global__ void copy_u32_kernel(const uint32_t* a, uint32_t* b, uint64_t n) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    b[i] = a[i];
}

// ---------------------------------------------------------------------------
// Visit: reverse lists

// Visit of a streamlined range [lo, hi).  An entry (o -> t) is a new
// reverse link of t when an earlier Visit of o recorded it and t has not
// been visited since (kFlagRevNew), or when o is in the range and the entry
// is new (recorded by this Visit).

FGIM_DEV bool link_is_new(uint32_t fl, uint64_t o, uint64_t lo, uint64_t hi) {
  return (fl & kFlagRevNew) || (o >= lo && o < hi && (fl & kFlagNew));
}

// reverse-segment sizes of the range's vertices: 2t new links, 2t+1 other
// in-edges (cnt zero on entry)
__global__ void rev_count_range_kernel(const uint64_t* keys, const uint32_t* flags, uint64_t nk, uint32_t k,
                                       uint64_t lo, uint64_t hi, uint32_t* cnt) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < nk;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint64_t kk = keys[i];
    if (kk == kSentinel) continue;
    const uint32_t t = key_id(kk);
    if (t < lo || t >= hi) continue;
    atomicAdd(&cnt[2u * t + (link_is_new(flags[i], i / k, lo, hi) ? 0u : 1u)], 1u);
  }
}

// A range vertex is active when its Cn is not empty (a new list entry or a
// new reverse link); an inactive one forms no pair, so its other in-edges
// are not placed.  Vertices outside the range are inactive.
__global__ void rev_active_range_kernel(const uint32_t* flags, uint64_t N, uint32_t k, uint64_t lo, uint64_t hi,
                                        uint32_t* cnt, uint32_t* active) {
  for (uint64_t v = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; v < N;
       v += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    bool act = false;
    if (v >= lo && v < hi) {
      act = cnt[2 * v] > 0;
      for (uint32_t e = 0; e < k && !act; ++e) act = (flags[v * k + e] & kFlagNew) != 0;
      if (!act) cnt[2 * v + 1] = 0u;
    }
    active[v] = act ? 1u : 0u;
  }
}

// reverse entries of the range's vertices; then the range's vertices
// consume their new links, and the range's new entries pointing outside it
// are recorded as new links of their targets
__global__ void rev_scatter_range_kernel(const uint64_t* keys, uint32_t* flags, uint64_t nk, uint32_t k,
                                         uint64_t lo, uint64_t hi, const uint32_t* active, uint32_t* cur,
                                         uint64_t* rev) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < nk;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint64_t kk = keys[i];
    if (kk == kSentinel) continue;
    const uint32_t t = key_id(kk);
    const uint64_t o = i / k;
    const uint32_t fl = flags[i];
    if (t >= lo && t < hi) {
      const bool isnew = link_is_new(fl, o, lo, hi);
      if (isnew || active[t]) {
        const uint32_t pos = atomicAdd(&cur[2u * t + (isnew ? 0u : 1u)], 1u);
        rev[pos] = (kk & 0xFFFFFFFF00000000ull) | static_cast<uint32_t>(o);
      }
      if (fl & kFlagRevNew) flags[i] = fl & ~static_cast<uint32_t>(kFlagRevNew);
    } else if (o >= lo && o < hi && (fl & kFlagNew)) {
      flags[i] = fl | kFlagRevNew;
    }
  }
}

// ---------------------------------------------------------------------------
// Update: the local join

struct JoinArgs {
  const float* X;
  uint64_t ld;
  uint32_t nc;
  int metric;
  uint64_t N;
  uint32_t k;
  uint32_t k_rev;
  const uint64_t* keys;      // snapshot lists
  const uint32_t* flags;     // flags before this round's Visit
  const uint32_t* rev_off;   // 2N+1
  const uint64_t* rev;       // reverse entries
  const uint64_t* sub_off;   // h offsets
  uint32_t h;
  uint32_t cap;              // capacity of the proposal buffer
  uint32_t* ptotal;          // proposals emitted (may exceed cap)
  uint32_t* ptgt;
  uint64_t* pkey;
  uint32_t P, M;
  uint32_t ccap;             // max |Cn| + |Co| = 2 (k + k_rev)
  int stage_rows;            // candidate rows copied to LDS
  // MFMA join
  const float* nrm2;         // squared FP32 norm of every base row
  const float* qerr2;        // squared norm of each row's BF16 rounding residual
  const uint16_t* xb;        // BF16 copy (dense rows of dim) or null: convert X
  uint32_t dim;
  uint32_t dpad;             // dim rounded up to 32 (MFMA K)
  uint32_t slice;            // dimensions staged in LDS at a time (multiple of 32)
  uint32_t* rechecked;       // pairs re-scored in FP32 after the screen
  // candidate sets of the MFMA join, built by cand_kernel
  uint32_t* cand;            // (u_hi - u_lo) x kMfmaMaxC: Cn then Co, each ascending
  uint32_t* ccnt;            // 2 (u_hi - u_lo): |Cn|, |Co|
  struct CandAux* aux;       // N: per-vertex screen data
  uint64_t* pairs;           // pairs passing the screen: (Cn id) | (partner id) << 32
  unsigned long long* npairs;      // pairs emitted this round (may exceed pair_cap; 64-bit: no wrap)
  unsigned long long* npairs_max;  // largest npairs over the rounds
  uint32_t pair_cap;
  uint64_t u_lo, u_hi;       // the vertices this Visit + Update covers
};

// per-vertex data the MFMA screen reads for every candidate
struct CandAux {
  uint64_t worst;  // key of the list's last entry (kSentinel while the list has a free slot)
  float nrm2;      // squared FP32 norm of the row
  float qerr;      // norm of the row's BF16 rounding residual, inflated by its own rounding bound
};

FGIM_DEV CandAux make_aux(uint64_t worst, float nrm2, float qerr2, float gam) {
  CandAux x;
  x.worst = worst;
  x.nrm2 = nrm2;
  x.qerr = sqrtf(qerr2) * (1.0f + gam) * 1.0001f;
  return x;
}

// top-k_rev of a reverse segment by key, appended to list (ids) via counter
template <int NR>
FGIM_DEV void rev_top(const uint64_t* seg, uint32_t len, uint32_t krev, uint32_t* list, uint32_t* cnt) {
  if (len <= krev) {
    for (uint32_t i = lane_id(); i < len; i += 64) list[atomicAdd(cnt, 1u)] = key_id(seg[i]);
    return;
  }
  Pool<NR> top;
  top.clear();
  for (uint32_t b = 0; b < len; b += 64) {
    const uint64_t ck = b + lane_id() < len ? seg[b + lane_id()] : kSentinel;
    top.insert_batch(ck, krev);
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const uint32_t e = r * 64 + lane_id();
    if (e < krev && top.key[r] != kSentinel) list[atomicAdd(cnt, 1u)] = key_id(top.key[r]);
  }
}

// Proposals of one vertex's join are staged in LDS and flushed to the global
// buffer with one atomic per vertex; a proposal that finds the stage full
// goes straight to the global buffer.
constexpr uint32_t kPropStage = 512;

FGIM_DEV void stage_proposal(const JoinArgs& a, uint32_t tgt, uint64_t key, uint32_t* lds_cnt, uint32_t* stgt,
                             uint64_t* skey) {
  const uint32_t pos = atomicAdd(lds_cnt, 1u);
  if (pos < kPropStage) {
    stgt[pos] = tgt;
    skey[pos] = key;
  } else {
    const uint32_t g = atomicAdd(a.ptotal, 1u);
    if (g < a.cap) {
      a.ptgt[g] = tgt;
      a.pkey[g] = key;
    }
  }
}

// sort ids[0..n) by sub-index (stable) into out, with their sub-indexes
FGIM_DEV void sort_by_sub(const uint32_t* ids, uint32_t n, const uint64_t* sub_off, uint32_t h, uint32_t* out,
                          uint32_t* gout, uint32_t* gtmp) {
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) gtmp[i] = sub_of(sub_off, h, ids[i]);
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
    const uint32_t g = gtmp[i];
    uint32_t pos = 0;
    for (uint32_t j = 0; j < n; ++j) pos += (gtmp[j] < g) || (gtmp[j] == g && j < i);
    out[pos] = ids[i];
    gout[pos] = g;
  }
  __syncthreads();
}

template <int NR, int MMAX>
__global__ void __launch_bounds__(256) join_kernel(JoinArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const uint32_t C = a.ccap;
  uint32_t* arr_n = reinterpret_cast<uint32_t*>(smem);          // C
  uint32_t* arr_o = arr_n + C;                                  // C
  uint32_t* cid = arr_o + C;                                    // C: Cn then Co, each sorted by sub-index
  uint32_t* cg = cid + C;                                       // sub-index of cid
  uint64_t* cw = reinterpret_cast<uint64_t*>(cg + C);           // worst key of cid's list
  uint32_t* counters = reinterpret_cast<uint32_t*>(cw + C);     // 8
  uint64_t* skey = reinterpret_cast<uint64_t*>(counters + 8);   // kPropStage
  uint32_t* stgt = reinterpret_cast<uint32_t*>(skey + kPropStage);
  float* rows = reinterpret_cast<float*>(stgt + kPropStage);    // C x (d + 4) (optional)
  const uint32_t d = a.nc * 4 + 4;  // padded LDS row stride (spreads rows over banks)
  const int wave = threadIdx.x / 64;
  const int P = static_cast<int>(a.P);
  const int M = static_cast<int>(a.M);
  const int l = threadIdx.x % P;

  for (uint64_t u = a.u_lo + blockIdx.x; u < a.u_hi; u += gridDim.x) {
    if (threadIdx.x < 8) counters[threadIdx.x] = 0;
    __syncthreads();
    // forward entries split by flag
    for (uint32_t t = threadIdx.x; t < a.k; t += 256) {
      const uint64_t kk = a.keys[u * a.k + t];
      if (kk == kSentinel) continue;
      if (a.flags[u * a.k + t] & kFlagNew) arr_n[atomicAdd(&counters[0], 1u)] = key_id(kk);
      else arr_o[atomicAdd(&counters[1], 1u)] = key_id(kk);
    }
    // reverse entries, cut to k_rev by key
    if (wave < 2) {
      const uint32_t seg = 2u * static_cast<uint32_t>(u) + wave;
      const uint32_t b0 = a.rev_off[seg], b1 = a.rev_off[seg + 1];
      rev_top<NR>(a.rev + b0, b1 - b0, a.k_rev, wave == 0 ? arr_n : arr_o, &counters[wave]);
    }
    __syncthreads();
    const uint32_t nn0 = counters[0], no0 = counters[1];
    // Cn: unique ids of arr_n (kept in arr_n's first slots via cid scratch)
    for (uint32_t i = threadIdx.x; i < nn0; i += 256) {
      const uint32_t v = arr_n[i];
      bool dup = false;
      for (uint32_t j = 0; j < i && !dup; ++j) dup = arr_n[j] == v;
      if (!dup) cid[atomicAdd(&counters[2], 1u)] = v;
    }
    __syncthreads();
    const uint32_t nn = counters[2];
    // Co: unique ids of arr_o that are not in Cn
    for (uint32_t i = threadIdx.x; i < no0; i += 256) {
      const uint32_t v = arr_o[i];
      bool dup = false;
      for (uint32_t j = 0; j < i && !dup; ++j) dup = arr_o[j] == v;
      for (uint32_t j = 0; j < nn && !dup; ++j) dup = cid[j] == v;
      if (!dup) cid[nn + atomicAdd(&counters[3], 1u)] = v;
    }
    __syncthreads();
    const uint32_t no = counters[3];
    const uint32_t c = nn + no;
    // order Cn and Co by sub-index: the partners of a Cn entry are then at
    // most three contiguous ranges
    for (uint32_t i = threadIdx.x; i < c; i += 256) arr_n[i] = cid[i];
    __syncthreads();
    sort_by_sub(arr_n, nn, a.sub_off, a.h, cid, cg, arr_o);
    sort_by_sub(arr_n + nn, no, a.sub_off, a.h, cid + nn, cg + nn, arr_o);
    for (uint32_t i = threadIdx.x; i < c; i += 256)
      cw[i] = a.keys[static_cast<uint64_t>(cid[i]) * a.k + a.k - 1];
    if (a.stage_rows) {
      for (uint32_t i = threadIdx.x; i < c * a.nc; i += 256) {
        const uint32_t e = i / a.nc, ch = i - e * a.nc;
        *reinterpret_cast<float4*>(rows + e * d + 4 * ch) =
            *reinterpret_cast<const float4*>(a.X + static_cast<uint64_t>(cid[e]) * a.ld + 4 * ch);
      }
    }
    __syncthreads();
    // Each P-lane group takes Cn rows i (dealt statically) and scores the
    // partners j: Cn entries past i's run of equal sub-index, and Co entries
    // of another sub-index.  Loops that contain cross-lane shuffles are
    // wave-uniform: they run to the wave's largest partner count, predicated
    // per group.
    {
      const uint32_t G = 64 / P, g = (threadIdx.x % 64) / P;
      for (uint32_t rbase = wave * G; rbase < nn; rbase += 4 * G) {
        const uint32_t i = rbase + g;
        const bool act = i < nn;
        uint32_t cn_hi = 0, co_lo = nn, co_hi = nn, n1 = 0, n2 = 0, n3 = 0;
        if (act) {
          const uint32_t gi = cg[i];
          cn_hi = i + 1;
          while (cn_hi < nn && cg[cn_hi] == gi) ++cn_hi;
          while (co_lo < c && cg[co_lo] < gi) ++co_lo;
          co_hi = co_lo;
          while (co_hi < c && cg[co_hi] == gi) ++co_hi;
          n1 = nn - cn_hi;
          n2 = co_lo - nn;
          n3 = c - co_hi;
        }
        const uint32_t total = n1 + n2 + n3;
        uint32_t tmax = total;
#pragma unroll
        for (int st = 32; st >= 1; st /= 2) tmax = max(tmax, static_cast<uint32_t>(__shfl_xor(static_cast<int>(tmax), st, 64)));
        float4 x[MMAX];
        const float* xr = a.stage_rows ? rows + (act ? i : 0u) * d : a.X + static_cast<uint64_t>(cid[act ? i : 0u]) * a.ld;
        load_row<MMAX>(x, xr, a.nc, P, M, l);
        const uint32_t vi = act ? cid[i] : 0u;
        const uint64_t wi = act ? cw[i] : 0ull;
        for (uint32_t t = 0; t < tmax; ++t) {
          const bool valid = t < total;
          const uint32_t j = !valid ? 0u : (t < n1 ? cn_hi + t : (t < n1 + n2 ? nn + (t - n1) : co_hi + (t - n1 - n2)));
          const float* rb = a.stage_rows ? rows + j * d : a.X + static_cast<uint64_t>(cid[j]) * a.ld;
          const float dd = pair_distance_x<MMAX>(x, rb, a.metric, a.nc, P, M, l, valid);
          if (valid && l == 0) {
            const uint32_t vj = cid[j];
            const uint64_t to_i = make_key(dd, vj), to_j = make_key(dd, vi);
            if (to_i < wi) stage_proposal(a, vi, to_i, &counters[4], stgt, skey);
            if (to_j < cw[j]) stage_proposal(a, vj, to_j, &counters[4], stgt, skey);
          }
        }
      }
    }
    // flush the stage with one global atomic
    __syncthreads();
    const uint32_t ns = min(counters[4], kPropStage);
    if (threadIdx.x == 0 && ns) counters[5] = atomicAdd(a.ptotal, ns);
    __syncthreads();
    const uint32_t base = counters[5];
    for (uint32_t t = threadIdx.x; t < ns; t += 256) {
      const uint32_t pos = base + t;
      if (pos < a.cap) {
        a.ptgt[pos] = stgt[t];
        a.pkey[pos] = skey[t];
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Update on MFMA: the neighbour x neighbour tile of each vertex is scored
// with v_mfma_f32_16x16x32_bf16 on BF16 copies of the candidate rows staged
// in LDS, every cross-sub-index pair is screened with a rigorous error
// margin, and the pairs that could still be a proposal are re-scored in
// canonical FP32.  The screen only skips pairs that provably cannot beat
// either end's worst entry, so the proposals are exactly those of the
// plain join.

// per row: squared FP32 norm and squared norm of the BF16 rounding residual
// x - bf16(x) (one wavefront per row)
__global__ void __launch_bounds__(256) row_norms_kernel(const float* X, uint64_t n, uint32_t dim, uint64_t ld,
                                                        float* out, float* qerr) {
  const uint32_t wave = threadIdx.x / 64;
  for (uint64_t row = blockIdx.x * 4ull + wave; row < n; row += gridDim.x * 4ull) {
    float s = 0.0f, q = 0.0f;
    for (uint32_t t = lane_id(); t < dim; t += 64) {
      const float x = X[row * ld + t];
      const float r = x - bf16_value(x);
      s = __builtin_fmaf(x, x, s);
      q = __builtin_fmaf(r, r, q);
    }
    for (int st = 32; st >= 1; st /= 2) {
      s += shfl_xor_f(s, st);
      q += shfl_xor_f(q, st);
    }
    if (lane_id() == 0) {
      out[row] = s;
      qerr[row] = q;
    }
  }
}

hipError_t launch_row_norms(const float* X, uint64_t n, uint32_t dim, uint64_t ld, float* nrm2, float* qerr2,
                            hipStream_t s) {
  const uint64_t b = (n + 3) / 4;
  hipLaunchKernelGGL(row_norms_kernel, dim3(static_cast<uint32_t>(std::min<uint64_t>(std::max<uint64_t>(b, 1), 65536))),
                     dim3(256), 0, s, X, n, dim, ld, nrm2, qerr2);
  return hipGetLastError();
}

constexpr uint32_t kMfmaMaxC = 128;       // candidates per vertex on the MFMA path
constexpr uint32_t kMfmaMaxCn = 64;       // |Cn| bound on the MFMA path (k + k_rev <= 64)
constexpr uint32_t kMfmaTilesPerWave = 7; // ceil(26 tile pairs / 4 waves) for |Cn| <= 64, c <= 128
constexpr uint32_t kPairChunk = 1024;     // pair-buffer slots a join workgroup claims at a time
constexpr uint64_t kPairBudget = 1ull << 28;  // pair-buffer entries (2 GiB) an Update chunk may use
constexpr uint64_t kNoPair = ~0ull;       // an unused pair-buffer slot
constexpr uint32_t kJoinStage = 4;  // row chunks a thread gathers before storing them

// position of the r-th set bit (r < popcount) of the 128-bit mask (m0, m1)
FGIM_DEV uint32_t select_bit(uint64_t m0, uint64_t m1, uint32_t r) {
  uint32_t pos = 0;
  uint64_t m = m0;
  const uint32_t c0 = static_cast<uint32_t>(__popcll(m0));
  if (r >= c0) {
    r -= c0;
    m = m1;
    pos = 64;
  }
#pragma unroll
  for (uint32_t w = 32; w >= 1; w >>= 1) {
    const uint64_t low = m & ((1ull << w) - 1ull);
    const uint32_t c = static_cast<uint32_t>(__popcll(low));
    if (r >= c) {
      r -= c;
      m >>= w;
      pos += w;
    }
  }
  return pos;
}

// bitonic sort of 64 uint32 values, one per lane, ascending
FGIM_DEV uint32_t wave_sort64(uint32_t v) {
  const uint32_t lane = static_cast<uint32_t>(lane_id());
#pragma unroll
  for (uint32_t k = 2; k <= 64; k <<= 1) {
#pragma unroll
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      const uint32_t o = static_cast<uint32_t>(__shfl_xor(static_cast<int>(v), static_cast<int>(j), 64));
      const bool lower = (lane & j) == 0;
      const bool asc = (lane & k) == 0;
      v = (lower == asc) ? min(v, o) : max(v, o);
    }
  }
  return v;
}

// bitonic sort of one 64-bit key per lane, ascending
FGIM_DEV uint64_t wave_sort64_keys(uint64_t v) {
  const uint32_t lane = static_cast<uint32_t>(lane_id());
#pragma unroll
  for (uint32_t k = 2; k <= 64; k <<= 1) {
#pragma unroll
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      const uint64_t o = shfl64(v, static_cast<int>(lane ^ j));
      const bool lower = (lane & j) == 0;
      const bool asc = (lane & k) == 0;
      v = (lower == asc) ? (o < v ? o : v) : (o > v ? o : v);
    }
  }
  return v;
}

// the 64 smallest of two ascending 64-key waves, ascending: lane l's
// min(a[l], b[63 - l]) forms a bitonic sequence of exactly those keys, which
// six half-cleaning steps sort
FGIM_DEV uint64_t wave_merge_low64(uint64_t a, uint64_t b) {
  const uint32_t lane = static_cast<uint32_t>(lane_id());
  const uint64_t br = shfl64(b, static_cast<int>(63u - lane));
  uint64_t v = a < br ? a : br;
#pragma unroll
  for (uint32_t j = 32; j > 0; j >>= 1) {
    const uint64_t o = shfl64(v, static_cast<int>(lane ^ j));
    v = (lane & j) == 0 ? (o < v ? o : v) : (o > v ? o : v);
  }
  return v;
}

// the unique non-NONE values of the sorted wave (one per lane) written to
// out in order; returns their count (wave-uniform)
FGIM_DEV uint32_t wave_unique64(uint32_t v, uint32_t* out) {
  const uint32_t prev = static_cast<uint32_t>(__shfl(static_cast<int>(v), lane_id() == 0 ? 0 : lane_id() - 1, 64));
  const bool keep = v != kNone && (lane_id() == 0 || v != prev);
  const uint64_t m = ballot(keep);
  if (keep) out[mbcnt(m)] = v;
  return static_cast<uint32_t>(popc64(m));
}

// Visit for the MFMA join, one vertex u per wavefront (four independent
// wavefronts per workgroup): Cn(u) = the new forward entries and the k_rev
// closest new reverse entries, Co(u) = the old ones not in Cn, each unique
// and ascending (ascending ids group by sub-index); written to a.cand /
// a.ccnt with u's own screen data.  k + k_rev <= 64, so each set fits one
// value per lane.
__global__ void __launch_bounds__(256) cand_kernel(JoinArgs a) {
  __shared__ uint32_t s_n[4][kMfmaMaxCn], s_o[4][kMfmaMaxCn], s_c[4][kMfmaMaxC];
  const int wave = threadIdx.x / 64;
  const int lane = lane_id();
  uint32_t* arr_n = s_n[wave];
  uint32_t* arr_o = s_o[wave];
  uint32_t* cid = s_c[wave];
  const float gam = fp32_gamma(a.dim);
  for (uint64_t u = a.u_lo + blockIdx.x * 4ull + wave; u < a.u_hi; u += gridDim.x * 4ull) {
    // u's list, the bounds of its two reverse segments and its screen data
    // are independent loads, issued together
    const bool in = static_cast<uint32_t>(lane) < a.k;
    const uint64_t kk = in ? a.keys[u * a.k + lane] : kSentinel;
    const uint32_t fl = in ? a.flags[u * a.k + lane] : 0u;
    // segment bounds are wave-uniform (readfirstlane): the selection below
    // loops over them with cross-lane steps
    const uint32_t o0 = uniform(a.rev_off[2 * u]), o1 = uniform(a.rev_off[2 * u + 1]),
                   o2 = uniform(a.rev_off[2 * u + 2]);
    const float nrm = lane == 0 ? a.nrm2[u] : 0.0f, qe2 = lane == 0 ? a.qerr2[u] : 0.0f;
    const uint32_t len[2] = {o1 - o0, o2 - o1};
    const uint32_t off[2] = {o0, o1};
    // the first 64 entries of both reverse segments
    uint64_t first[2];
#pragma unroll
    for (int kind = 0; kind < 2; ++kind)
      first[kind] = static_cast<uint32_t>(lane) < len[kind] ? a.rev[off[kind] + lane] : kSentinel;
    // forward entries, split by flag
    const bool valid = kk != kSentinel;
    const bool isnew = valid && (fl & kFlagNew);
    const uint64_t mn = ballot(isnew), mo = ballot(valid && !isnew);
    if (isnew) arr_n[mbcnt(mn)] = key_id(kk);
    if (valid && !isnew) arr_o[mbcnt(mo)] = key_id(kk);
    uint32_t cnt[2] = {static_cast<uint32_t>(popc64(mn)), static_cast<uint32_t>(popc64(mo))};
    const uint64_t wk = readlane64(kk, static_cast<int>(a.k - 1));
    if (lane == 0) a.aux[u] = make_aux(wk, nrm, qe2, gam);
    // the k_rev closest reverse entries of each kind, appended by ballot
#pragma unroll
    for (int kind = 0; kind < 2; ++kind) {
      uint32_t* list = kind == 0 ? arr_n : arr_o;
      uint64_t pick = first[kind];
      if (len[kind] > a.k_rev) {
        // the k_rev smallest keys (unique: one per owner) by sorting 64 at a
        // time and keeping the 64 smallest (k_rev < 64 here), whatever order
        // the segment holds them in
        uint64_t top = wave_sort64_keys(first[kind]);
        for (uint32_t b = 64; b < len[kind]; b += 64) {
          const uint64_t ck = b + lane < len[kind] ? a.rev[off[kind] + b + lane] : kSentinel;
          top = wave_merge_low64(top, wave_sort64_keys(ck));
        }
        pick = static_cast<uint32_t>(lane) < a.k_rev ? top : kSentinel;
      }
      const bool take = pick != kSentinel;
      const uint64_t mt = ballot(take);
      if (take) list[cnt[kind] + mbcnt(mt)] = key_id(pick);
      cnt[kind] += static_cast<uint32_t>(popc64(mt));
    }
    // no new candidate: no pair, so no set (the join skips the vertex)
    if (cnt[0] == 0) {
      if (lane == 0) {
        a.ccnt[2 * (u - a.u_lo)] = 0;
        a.ccnt[2 * (u - a.u_lo) + 1] = 0;
      }
      continue;
    }
    wave_lds_sync();
    // Cn: sorted unique new ids
    const uint32_t cn = cnt[0], co = cnt[1];
    const uint32_t vn = wave_sort64(static_cast<uint32_t>(lane) < cn ? arr_n[lane] : kNone);
    const uint32_t nn = wave_unique64(vn, cid);
    // Co: sorted unique old ids that are not in Cn
    const uint32_t vo = wave_sort64(static_cast<uint32_t>(lane) < co ? arr_o[lane] : kNone);
    wave_lds_sync();
    const uint32_t prev = static_cast<uint32_t>(__shfl(static_cast<int>(vo), lane == 0 ? 0 : lane - 1, 64));
    bool keep = vo != kNone && (lane == 0 || vo != prev);
    if (keep) {
      uint32_t lo = 0, hi = nn;
      while (lo < hi) {
        const uint32_t mid = (lo + hi) / 2;
        if (cid[mid] < vo) lo = mid + 1;
        else hi = mid;
      }
      keep = !(lo < nn && cid[lo] == vo);
    }
    const uint64_t mk = ballot(keep);
    if (keep) cid[nn + mbcnt(mk)] = vo;
    const uint32_t no = static_cast<uint32_t>(popc64(mk));
    wave_lds_sync();
    for (uint32_t i = lane; i < nn + no; i += 64) a.cand[(u - a.u_lo) * kMfmaMaxC + i] = cid[i];
    if (lane == 0) {
      a.ccnt[2 * (u - a.u_lo)] = nn;
      a.ccnt[2 * (u - a.u_lo) + 1] = no;
    }
    wave_lds_sync();
  }
}

__global__ void __launch_bounds__(256) join_mfma_kernel(JoinArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  uint64_t* cw = reinterpret_cast<uint64_t*>(smem);              // worst key of each candidate's list
  uint64_t* pmask = cw + kMfmaMaxC;                               // 64 x 2 words: passing partners of Cn row i
  uint32_t* cid = reinterpret_cast<uint32_t*>(pmask + 2 * kMfmaMaxCn); // 128: Cn then Co, ascending id
  uint32_t* cg = cid + kMfmaMaxC;                                 // sub-index
  float* cnrm = reinterpret_cast<float*>(cg + kMfmaMaxC);         // squared norms
  float* cqe = cnrm + kMfmaMaxC;                                  // BF16 residual norms
  uint32_t* rowoff = reinterpret_cast<uint32_t*>(cqe + kMfmaMaxC); // 65 prefix counts
  uint32_t* counters = rowoff + 68;  // 16: [0..7] per vertex; [8..10] pair chunk base, used, size
  uint16_t* brows = reinterpret_cast<uint16_t*>(counters + 16);   // BF16 slices, 128 x (slice + 8)
  const uint32_t srow = a.slice + 8;
  const int wave = threadIdx.x / 64;
  const int lane = lane_id();
  const float gam = fp32_gamma(a.dim);
  uint32_t nrech = 0;  // pairs passing the screen (thread 0)
  if (threadIdx.x >= 8 && threadIdx.x < 16) counters[threadIdx.x] = 0;

  // The next vertex's candidate ids load while the current one is screened,
  // and their screen records after its MFMA tiles: thread t < 128 holds
  // candidate t.
  uint32_t pf_n = 0, pf_o = 0, pf_v = kNone;
  CandAux pf_x{};
  auto fetch_ids = [&](uint64_t w) {
    if (w < a.u_hi) {
      pf_n = a.ccnt[2 * (w - a.u_lo)];
      pf_o = a.ccnt[2 * (w - a.u_lo) + 1];
      pf_v = threadIdx.x < kMfmaMaxC ? a.cand[(w - a.u_lo) * kMfmaMaxC + threadIdx.x] : kNone;
    }
  };
  auto fetch_aux = [&]() {
    if (threadIdx.x < pf_n + pf_o) pf_x = a.aux[pf_v];
  };
  fetch_ids(a.u_lo + blockIdx.x);
  fetch_aux();

  for (uint64_t u = a.u_lo + blockIdx.x; u < a.u_hi; u += gridDim.x) {
    if (threadIdx.x < 8) counters[threadIdx.x] = 0;
    if (threadIdx.x < kMfmaMaxC) pmask[threadIdx.x] = 0;
    const uint32_t nn = uniform(pf_n), no = uniform(pf_o);
    const uint32_t c = nn + no;
    if (threadIdx.x < c) {
      cid[threadIdx.x] = pf_v;
      cg[threadIdx.x] = sub_of(a.sub_off, a.h, pf_v);
      cw[threadIdx.x] = pf_x.worst;
      cnrm[threadIdx.x] = pf_x.nrm2;
      cqe[threadIdx.x] = pf_x.qerr;
    }
    fetch_ids(u + gridDim.x);
    __syncthreads();
    const uint32_t nI = (nn + 15) / 16, nC = (c + 15) / 16;
    uint32_t T = 0;
    for (uint32_t I = 0; I < nI; ++I) T += nC - I;
    floatx4_t acc[kMfmaTilesPerWave];
#pragma unroll
    for (uint32_t t = 0; t < kMfmaTilesPerWave; ++t) acc[t] = floatx4_t{0.f, 0.f, 0.f, 0.f};
    // BF16 slices of the dimensions through LDS (none when the vertex has
    // no new candidate: then it has no tile and no pair; T is uniform)
    for (uint32_t s0 = 0; T > 0 && s0 < a.dpad; s0 += a.slice) {
      const uint32_t sw = min(a.slice, a.dpad - s0);   // multiple of 32
      __syncthreads();
      const uint32_t per_row = sw / 8;
      const uint32_t total = nC * 16 * per_row;
      // kJoinStage chunks per thread are gathered before any is stored, so
      // their memory latencies overlap (one wait per batch, not per chunk)
      for (uint32_t base = 0; base < total; base += 256 * kJoinStage) {
        shortx8_t v8[kJoinStage];
#pragma unroll
        for (uint32_t b = 0; b < kJoinStage; ++b) {
          const uint32_t idx = base + b * 256 + threadIdx.x;
          const uint32_t e = idx / per_row, q = idx - e * per_row;
          const uint32_t t0 = s0 + 8 * q;
          v8[b] = shortx8_t{0, 0, 0, 0, 0, 0, 0, 0};
          if (idx < total && e < c && t0 < a.dim) {
            const uint64_t v = cid[e];
            if (a.xb) {
              v8[b] = *reinterpret_cast<const shortx8_t*>(a.xb + v * a.dim + t0);
            } else {
              const float4 f0 = *reinterpret_cast<const float4*>(a.X + v * a.ld + t0);
              const float4 f1 = t0 + 4 < a.dim ? *reinterpret_cast<const float4*>(a.X + v * a.ld + t0 + 4)
                                               : make_float4(0.f, 0.f, 0.f, 0.f);
              v8[b][0] = bf16_rne(f0.x); v8[b][1] = bf16_rne(f0.y); v8[b][2] = bf16_rne(f0.z); v8[b][3] = bf16_rne(f0.w);
              v8[b][4] = bf16_rne(f1.x); v8[b][5] = bf16_rne(f1.y); v8[b][6] = bf16_rne(f1.z); v8[b][7] = bf16_rne(f1.w);
            }
          }
        }
#pragma unroll
        for (uint32_t b = 0; b < kJoinStage; ++b) {
          const uint32_t idx = base + b * 256 + threadIdx.x;
          const uint32_t e = idx / per_row, q = idx - e * per_row;
          if (idx < total) *reinterpret_cast<shortx8_t*>(brows + e * srow + 8 * q) = v8[b];
        }
      }
      __syncthreads();
#pragma unroll
      for (uint32_t sl = 0; sl < kMfmaTilesPerWave; ++sl) {
        uint32_t tp = static_cast<uint32_t>(wave) + 4u * sl;
        if (tp >= T) break;
        uint32_t I = 0;
        while (tp >= nC - I) {
          tp -= nC - I;
          ++I;
        }
        const uint32_t J = I + tp;
        for (uint32_t kb = 0; kb < sw; kb += 32) {
          const shortx8_t ra = *reinterpret_cast<const shortx8_t*>(brows + (16 * I + lane % 16) * srow + kb + 8 * (lane / 16));
          const shortx8_t rb = *reinterpret_cast<const shortx8_t*>(brows + (16 * J + lane % 16) * srow + kb + 8 * (lane / 16));
          acc[sl] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, ra),
                                                            __builtin_bit_cast(bf16x8_t, rb), acc[sl], 0, 0, 0);
        }
      }
    }
    fetch_aux();
    // Screen (screen_estimate): a pair passes when its estimate minus the
    // bound could still beat the worst entry of either end.
#pragma unroll
    for (uint32_t sl = 0; sl < kMfmaTilesPerWave; ++sl) {
      uint32_t tp = static_cast<uint32_t>(wave) + 4u * sl;
      if (tp >= T) break;
      uint32_t I = 0;
      while (tp >= nC - I) {
        tp -= nC - I;
        ++I;
      }
      const uint32_t J = I + tp;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const uint32_t i = 16 * I + 4 * (lane / 16) + r, j = 16 * J + lane % 16;
        const bool valid = i < nn && j < c && j > i && cg[i] != cg[j];
        if (!valid) continue;
        float dt, err;
        screen_estimate(acc[sl][r], cnrm[i], cnrm[j], cqe[i], cqe[j], gam, a.metric, &dt, &err);
        const float thr = fmaxf(key_dist(cw[i]), key_dist(cw[j]));
        if (dt - err <= thr)
          atomicOr(reinterpret_cast<unsigned long long*>(&pmask[2 * i + j / 64]), 1ull << (j % 64));
      }
    }
    __syncthreads();
    // prefix counts of passing partners per Cn row (one wave, nn <= 64)
    if (wave == 0) {
      const uint32_t cnt = static_cast<uint32_t>(lane) < nn
                               ? static_cast<uint32_t>(__popcll(pmask[2 * lane]) + __popcll(pmask[2 * lane + 1]))
                               : 0u;
      uint32_t incl = cnt;
#pragma unroll
      for (int st = 1; st < 64; st <<= 1) {
        const uint32_t o = static_cast<uint32_t>(__shfl_up(static_cast<int>(incl), st, 64));
        if (lane >= st) incl += o;
      }
      rowoff[lane + 1] = incl;
      if (lane == 0) rowoff[0] = 0;
    }
    __syncthreads();
    const uint32_t np = rowoff[nn];
    // the passing pairs go to the pair buffer, enumerated flat over all rows,
    // into chunks of it this workgroup claims (one global atomic per chunk,
    // not per vertex); recheck_kernel scores them exactly
    if (threadIdx.x == 0) {
      nrech += np;
      const uint32_t used = counters[9], size = counters[10];
      const uint32_t rem = size - used;
      counters[4] = counters[8] + used;  // first part: the current chunk's tail
      counters[5] = min(np, rem);
      if (np > rem) {  // second part: a new chunk
        const uint32_t need = np - rem;
        const uint32_t sz = max(kPairChunk, need);
        // a chunk past the buffer starts at pair_cap, so that every position
        // in it is dropped (and the 32-bit positions cannot wrap)
        const unsigned long long b64 = atomicAdd(a.npairs, static_cast<unsigned long long>(sz));
        counters[8] = b64 < a.pair_cap ? static_cast<uint32_t>(b64) : a.pair_cap;
        counters[9] = need;
        counters[10] = sz;
        counters[6] = counters[8];
      } else {
        counters[9] = used + np;
      }
    }
    __syncthreads();
    const uint32_t p0 = counters[4], n0 = counters[5], p1 = counters[6];
    for (uint32_t idx = threadIdx.x; idx < np; idx += 256) {
      uint32_t lo = 0, hi = nn;  // the row holding idx: last row with rowoff <= idx
      while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) / 2;
        if (rowoff[mid] <= idx) lo = mid;
        else hi = mid;
      }
      const uint32_t jj = select_bit(pmask[2 * lo], pmask[2 * lo + 1], idx - rowoff[lo]);
      const uint64_t pos = idx < n0 ? static_cast<uint64_t>(p0) + idx : static_cast<uint64_t>(p1) + (idx - n0);
      if (pos < a.pair_cap) a.pairs[pos] = (static_cast<uint64_t>(cid[jj]) << 32) | cid[lo];
    }
    __syncthreads();
  }
  // the unused tail of the last chunk holds no pair
  const uint64_t t0 = static_cast<uint64_t>(counters[8]) + counters[9];
  const uint64_t t1 = static_cast<uint64_t>(counters[8]) + counters[10];
  for (uint64_t t = t0 + threadIdx.x; t < t1; t += 256)
    if (t < a.pair_cap) a.pairs[t] = kNoPair;
  if (threadIdx.x == 0 && nrech) atomicAdd(a.rechecked, nrech);
}

// Exact re-scoring of the pairs that passed the MFMA screen: one pair per
// group of P lanes, the canonical FP32 distance from the base rows, and a
// proposal to each end whose list's worst entry it beats.
constexpr uint32_t kRecheckStage = 2048;  // proposals staged in LDS per flush

template <int MMAX>
__global__ void __launch_bounds__(256) recheck_kernel(JoinArgs a) {
  __shared__ uint64_t skey[kRecheckStage];
  __shared__ uint32_t stgt[kRecheckStage];
  __shared__ uint32_t scount, sbase;
  const int P = static_cast<int>(a.P), M = static_cast<int>(a.M);
  const int l = threadIdx.x % P;
  const uint32_t per_block = 256 / P;
  const uint64_t demand = *a.npairs;
  const uint64_t n = demand < a.pair_cap ? demand : a.pair_cap;
  if (blockIdx.x == 0 && threadIdx.x == 0) atomicMax(a.npairs_max, static_cast<unsigned long long>(demand));
  if (threadIdx.x == 0) scount = 0;
  __syncthreads();
  // proposals are staged in LDS and flushed with one global atomic per
  // flush (a single shared counter would serialise on contention)
  auto flush = [&]() {
    const uint32_t ns = scount;
    if (threadIdx.x == 0 && ns) sbase = atomicAdd(a.ptotal, ns);
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < ns; t += 256) {
      const uint32_t pos = sbase + t;
      if (pos < a.cap) {
        a.ptgt[pos] = stgt[t];
        a.pkey[pos] = skey[t];
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) scount = 0;
    __syncthreads();
  };
  // R pairs per group and iteration: both ends' rows and worst keys of
  // every pair are loaded before any distance is reduced
  constexpr int R = MMAX <= 4 ? 2 : 1;
  const uint64_t step = static_cast<uint64_t>(per_block) * R;
  for (uint64_t b0 = static_cast<uint64_t>(blockIdx.x) * step; b0 < n; b0 += static_cast<uint64_t>(gridDim.x) * step) {
    uint64_t pr[R], wi[R], wj[R];
    bool act[R];
    float4 x[R][MMAX], y[R][MMAX];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint64_t idx = b0 + static_cast<uint64_t>(r) * per_block + threadIdx.x / P;
      pr[r] = idx < n ? a.pairs[idx] : kNoPair;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      act[r] = pr[r] != kNoPair;
      if (!act[r]) pr[r] = 0;
      const uint32_t vi = static_cast<uint32_t>(pr[r]), vj = static_cast<uint32_t>(pr[r] >> 32);
      load_row_chunks<MMAX>(x[r], a.X + static_cast<uint64_t>(vi) * a.ld, a.nc, P, M, l, act[r]);
      load_row_chunks<MMAX>(y[r], a.X + static_cast<uint64_t>(vj) * a.ld, a.nc, P, M, l, act[r]);
      wi[r] = wj[r] = 0;
      if (act[r] && l == 0) {
        wi[r] = a.aux[vi].worst;
        wj[r] = a.aux[vj].worst;
      }
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const float dd = chunks_distance<MMAX>(x[r], y[r], a.metric, a.nc, P, M, l, act[r]);
      if (act[r] && l == 0) {
        const uint32_t vi = static_cast<uint32_t>(pr[r]), vj = static_cast<uint32_t>(pr[r] >> 32);
        const uint64_t ki = make_key(dd, vj), kj = make_key(dd, vi);
        if (ki < wi[r]) {
          const uint32_t pos = atomicAdd(&scount, 1u);
          stgt[pos] = vi;
          skey[pos] = ki;
        }
        if (kj < wj[r]) {
          const uint32_t pos = atomicAdd(&scount, 1u);
          stgt[pos] = vj;
          skey[pos] = kj;
        }
      }
    }
    __syncthreads();
    if (scount + 2 * step > kRecheckStage) flush();
  }
  flush();
}

// ---------------------------------------------------------------------------
// proposals, grouped by target (group_records), applied

// first k of snapshot (old) U proposals (new), one entry per id; every
// list's new entries turn old.  The indegrees T and the counts of new
// in-edges follow the change: a dropped old entry lowers T, an accepted
// proposal raises T and the new count (newc is zero on entry).
template <int NR>
__global__ void __launch_bounds__(256) apply_kernel(uint64_t* keys, uint32_t* flags, uint64_t N, uint32_t k,
                                                    const uint32_t* poff, const uint64_t* sorted,
                                                    uint32_t* ptotal_max, const uint32_t* ptotal, uint32_t* T,
                                                    uint32_t* newc) {
  const uint64_t wave = blockIdx.x * 4ull + threadIdx.x / 64;
  const uint64_t nw = gridDim.x * 4ull;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    atomicMax(ptotal_max, *ptotal);
    atomicAdd(ptotal_max + 2, *ptotal);
  }
  for (uint64_t a = wave; a < N; a += nw) {
    Pool<NR> list;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const uint32_t e = r * 64 + lane_id();
      list.key[r] = e < k ? keys[a * k + e] : kSentinel;
    }
    list.exp = 0;
    uint64_t old[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) old[r] = list.key[r];
    const uint32_t b0 = poff[a], b1 = poff[a + 1];
    for (uint32_t b = b0; b < b1; b += 64) {
      const uint64_t ck = b + lane_id() < b1 ? sorted[b + lane_id()] : kSentinel;
      list.insert_batch(ck, k, 1u);
    }
    if (b1 > b0) {
      // an old entry is kept iff it is not beyond the new last entry
      const uint64_t last = list.theta(k);
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        if (old[r] != kSentinel && old[r] > last) atomicSub(&T[key_id(old[r])], 1u);
        if ((list.exp >> r) & 1u) {
          atomicAdd(&T[key_id(list.key[r])], 1u);
          atomicAdd(&newc[key_id(list.key[r])], 1u);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const uint32_t e = r * 64 + lane_id();
      if (e < k) {
        keys[a * k + e] = list.key[r];
        flags[a * k + e] = (list.exp >> r) & 1u;
      }
    }
  }
}

// Apply of one streamlined micro-batch, which visited the lists in
// [lo, hi): a list keeps the first k of its entries and the proposals to it,
// one entry per id.  Its surviving entries keep their flags (new, recorded
// link), except that the visited lists' entries are no longer new; accepted
// proposals are new.  T follows every change (the counts of new in-edges
// are not kept: streamlined Visits count links directly).  Lists outside
// the range without proposals do not change and are skipped.
template <int NR>
__global__ void __launch_bounds__(256) apply_stream_kernel(uint64_t* keys, uint32_t* flags, uint64_t N, uint32_t k,
                                                           uint64_t lo, uint64_t hi, const uint32_t* poff,
                                                           const uint64_t* sorted, uint32_t* ptotal_max,
                                                           const uint32_t* ptotal, uint32_t* T) {
  // the list index and its proposal bounds are wave-uniform (readfirstlane),
  // so the skip below is a uniform branch in a loop with cross-lane steps
  const uint64_t wave = uniform(blockIdx.x * 4u + threadIdx.x / 64u);
  const uint64_t nw = gridDim.x * 4ull;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    atomicMax(ptotal_max, *ptotal);
    atomicAdd(ptotal_max + 2, *ptotal);
  }
  for (uint64_t a = wave; a < N; a += nw) {
    const bool visited = a >= lo && a < hi;
    const uint32_t b0 = uniform(poff[a]), b1 = uniform(poff[a + 1]);
    if (!visited && b1 == b0) continue;
    Pool<NR> list;
    uint32_t fl[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const uint32_t e = r * 64 + lane_id();
      list.key[r] = e < k ? keys[a * k + e] : kSentinel;
      fl[r] = e < k ? (flags[a * k + e] & (kFlagNew | kFlagRevNew)) : 0u;
      // a visited list's new entries turn old
      if (visited) fl[r] &= ~static_cast<uint32_t>(kFlagNew);
    }
    list.exp = 0;
    uint64_t old[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) old[r] = list.key[r];
    for (uint32_t b = b0; b < b1; b += 64) {
      const uint64_t ck = b + lane_id() < b1 ? sorted[b + lane_id()] : kSentinel;
      list.insert_batch(ck, k, 1u);
    }
    if (b1 > b0) {
      // an old entry is kept iff it is not beyond the new last entry
      const uint64_t last = list.theta(k);
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        if (old[r] != kSentinel && old[r] > last) atomicSub(&T[key_id(old[r])], 1u);
        if ((list.exp >> r) & 1u) atomicAdd(&T[key_id(list.key[r])], 1u);
      }
    }
    // the kept entries of the list are its first entries, in order, so the
    // j-th entry that is not a proposal is the list's j-th entry
    uint32_t before = 0;
    uint32_t out[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const bool kept = !((list.exp >> r) & 1u);
      const uint64_t m = ballot(kept);
      const uint32_t j = before + mbcnt(m);
      before += static_cast<uint32_t>(popc64(m));
      uint32_t f = 0u;
#pragma unroll
      for (int q = 0; q < NR; ++q) {
        const uint32_t fq = static_cast<uint32_t>(__shfl(static_cast<int>(fl[q]), static_cast<int>(j % 64), 64));
        if (j / 64 == static_cast<uint32_t>(q)) f = fq;
      }
      out[r] = kept ? f : static_cast<uint32_t>(kFlagNew);
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const uint32_t e = r * 64 + lane_id();
      if (e < k) {
        keys[a * k + e] = list.key[r];
        flags[a * k + e] = list.key[r] == kSentinel ? 0u : out[r];
      }
    }
  }
}

// the screen data of every vertex from its current list (a streamlined
// micro-batch screens against the lists the earlier ones left)
__global__ void aux_refresh_kernel(const uint64_t* keys, uint64_t N, uint32_t k, const float* nrm2, const float* qerr2,
                                   uint32_t dim, CandAux* aux) {
  const float gam = fp32_gamma(dim);
  for (uint64_t u = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; u < N;
       u += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    aux[u] = make_aux(keys[u * k + k - 1], nrm2[u], qerr2[u], gam);
}

// reverse-list segment sizes of the next Visit from the maintained counts:
// 2v holds v's new in-edges, 2v+1 its old ones
// A vertex is active when its list holds a new entry or it has a new
// in-edge (a maintained count): otherwise its Cn is empty, its join forms no
// pair and reads no reverse entry, so its old reverse segment is left empty
// (the reverse lists of new entries are always complete).  A wave takes 64
// consecutive vertices, whose flags are 64 k consecutive words: it reads
// them 64 at a time (coalesced, eight loads in flight), and each lane tests
// the bits of the ballot that belong to its own vertex.  The result is one
// bit per vertex, written 64 at a time; every loop bound is wave-uniform.
__global__ void rev_active_kernel(const uint32_t* newc, const uint32_t* flags, uint32_t k, uint64_t N,
                                  uint32_t* active_bits) {
  constexpr uint32_t kIn = 8;
  const uint64_t nw = static_cast<uint64_t>(gridDim.x) * (blockDim.x / 64);
  const uint64_t wave = uniform(blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64);
  const uint32_t l = static_cast<uint32_t>(lane_id());
  const uint64_t nk = N * k;
  for (uint64_t base = wave * 64; base < N; base += nw * 64) {
    const uint64_t v = base + l;
    bool act = v < N && newc[v] > 0;
    const uint64_t w0 = base * k;  // first flag word of the block
    const uint32_t my_lo = l * k, my_hi = l * k + k;  // my vertex's words, block-relative
    for (uint32_t j0 = 0; j0 < k; j0 += kIn) {
      uint32_t f[kIn];
#pragma unroll
      for (uint32_t t = 0; t < kIn; ++t) {
        const uint64_t w = w0 + static_cast<uint64_t>(j0 + t) * 64 + l;
        f[t] = j0 + t < k && w < nk ? flags[w] : 0u;
      }
#pragma unroll
      for (uint32_t t = 0; t < kIn; ++t) {
        const uint64_t m = ballot((f[t] & kFlagNew) != 0u);
        const uint32_t c0 = (j0 + t) * 64;  // block-relative words of this row
        const uint32_t lo = my_lo > c0 ? my_lo : c0, hi = my_hi < c0 + 64 ? my_hi : c0 + 64;
        if (lo < hi) {
          const uint32_t len = hi - lo;
          const uint64_t bits = len == 64 ? ~0ull : ((1ull << len) - 1ull);
          act = act || ((m >> (lo - c0)) & bits) != 0ull;
        }
      }
    }
    const uint64_t mv = ballot(act);
    if (l == 0) active_bits[base >> 5] = static_cast<uint32_t>(mv);
    if (l == 32 && base + 32 < N) active_bits[(base >> 5) + 1] = static_cast<uint32_t>(mv >> 32);
  }
}

// ---------------------------------------------------------------------------
// indegree and repair

__global__ void indegree_kernel(const uint64_t* keys, uint64_t nk, uint32_t* T) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < nk;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint64_t kk = keys[i];
    if (kk != kSentinel) atomicAdd(&T[key_id(kk)], 1u);
  }
}

// zero-indegree vertices with a neighbour to try: a vertex whose own list is
// empty (a dropped one, or one no search reached) has no candidate, so its
// step could change nothing and is left out of the batches
__global__ void zero_mask_kernel(const uint32_t* T, const uint64_t* keys, uint32_t k, uint64_t N, uint32_t* mask) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < N;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    mask[i] = T[i] == 0u && keys[i * k] != kSentinel ? 1u : 0u;
}

// list of the zero-indegree vertices in ascending id, with the first key of
// each one's list (its closest neighbour; these lists never change during
// the repair pass)
__global__ void zero_compact_kernel(const uint32_t* mask, const uint32_t* off, uint64_t N, const uint64_t* keys,
                                    uint32_t k, uint32_t* zero, uint64_t* zkey) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < N;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    if (mask[i]) {
      zero[off[i]] = static_cast<uint32_t>(i);
      zkey[off[i]] = keys[i * k];
    }
}

// The repair runs in a single workgroup, so workgroup-scope coherence is
// all its waves need for the lists and indegrees they share.
FGIM_DEV uint64_t ld_wg64(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

FGIM_DEV uint32_t ld_wg32(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Algorithm 4.  Zero-indegree vertices v* are taken in ascending id; the
// neighbours v of v* are tried from the closest; in N(v) the farthest entry
// that is not marked replaced and whose indegree exceeds 1 is evicted (or a
// free slot is used), and v* enters N(v) at its sorted place, flagged new and
// replaced.  Lists of the v* themselves never change during the pass (no
// list holds a zero-indegree vertex before its own turn).
//
// The pass keeps this sequential order but runs speculatively, in batches of
// consecutive steps: every step makes its first attempt (the closest
// neighbour v) against the state at the batch start, all at once; then the
// batch commits its longest prefix in which no step read a list that an
// earlier step of the batch writes, or an indegree that earlier steps may
// lower to 1 or below.  A step writes N(v), T(v') of the entry v' it evicts
// (a decrement) and T(v*); it read N(v) and T of N(v)'s entries (and v*'s
// own list, which no step changes), and of those indegrees only the test
// "> 1" decides anything.  Earlier writes are looked up in two LDS hash
// tables that map a vertex to the first step of the batch writing its list
// or evicting it, the second with the batch's eviction count.  A step whose
// first attempt fails continues alone, as the first step of a batch.
// Committed steps therefore take exactly the decisions of the sequential
// loop, and reach its state.

// state read by one attempt (v = the neighbour of v* tried)
template <int NR>
struct Attempt {
  uint64_t lk[NR];
  uint32_t lf[NR];
  int drop;  // entry to evict, -1 for a free slot
  bool ok;   // v* can enter N(v)
};

// decide an attempt from N(v) (keys lk, flags lf) and the entries'
// indegrees tv
template <int NR>
FGIM_DEV void decide_attempt(Attempt<NR>& at, const uint32_t (&tv)[NR], uint32_t k) {
  uint64_t lastk = kSentinel;
#pragma unroll
  for (int r = 0; r < NR; ++r)
    if (static_cast<uint32_t>(r) == (k - 1) / 64) lastk = readlane64(at.lk[r], (k - 1) % 64);
  at.drop = -1;
  at.ok = true;
  if (lastk != kSentinel) {
    bool cand[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const uint32_t e = r * 64 + lane_id();
      cand[r] = e < k && !(at.lf[r] & kFlagReplaced) && tv[r] > 1u;
    }
#pragma unroll
    for (int r = NR - 1; r >= 0; --r) {
      const uint64_t m = ballot(cand[r]);
      if (at.drop < 0 && m) at.drop = r * 64 + 63 - __clzll(static_cast<long long>(m));
    }
    at.ok = at.drop >= 0;
  }
}

template <int NR>
FGIM_DEV Attempt<NR> try_neighbour(const uint64_t* keys, const uint32_t* flags, const uint32_t* T, uint32_t v,
                                   uint32_t k) {
  Attempt<NR> at;
  uint32_t tv[NR];
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const uint32_t e = r * 64 + lane_id();
    at.lk[r] = e < k ? ld_wg64(&keys[static_cast<uint64_t>(v) * k + e]) : kSentinel;
    at.lf[r] = e < k ? ld_wg32(&flags[static_cast<uint64_t>(v) * k + e]) : 0u;
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) tv[r] = at.lk[r] != kSentinel ? ld_wg32(&T[key_id(at.lk[r])]) : 0u;
  decide_attempt<NR>(at, tv, k);
  return at;
}

// write N(v) with entry `drop` removed (if any) and key nk inserted, and
// update the indegrees (the evicted entry's by an atomic decrement: other
// steps of a committed prefix may lower it too)
template <int NR>
FGIM_DEV void commit_attempt(uint64_t* keys, uint32_t* flags, uint32_t* T, uint32_t* newc, const Attempt<NR>& at,
                             uint32_t v, uint32_t vs, uint64_t nk, uint32_t k) {
  int pos = 0;
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int e = r * 64 + lane_id();
    pos += popc64(ballot(e != at.drop && at.lk[r] < nk));
  }
  uint64_t dk = kSentinel;
  uint32_t df = 0;
#pragma unroll
  for (int r = 0; r < NR; ++r)
    if (at.drop >= 0 && r == at.drop / 64) {
      dk = readlane64(at.lk[r], at.drop % 64);
      df = readlane(at.lf[r], at.drop % 64);
    }
  if (at.drop >= 0 && lane_id() == 0) {
    __hip_atomic_fetch_sub(&T[key_id(dk)], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (newc && (df & kFlagNew)) atomicSub(&newc[key_id(dk)], 1u);
  }
#pragma unroll
  for (int r = 0; r < NR; ++r) {
    const int e = r * 64 + lane_id();
    if (e >= static_cast<int>(k) || e == at.drop || at.lk[r] == kSentinel) continue;
    int ne = e - (at.drop >= 0 && e > at.drop ? 1 : 0);
    if (ne >= pos) ++ne;
    if (ne < static_cast<int>(k)) {
      keys[static_cast<uint64_t>(v) * k + ne] = at.lk[r];
      flags[static_cast<uint64_t>(v) * k + ne] = at.lf[r];
    }
  }
  if (lane_id() == 0) {
    keys[static_cast<uint64_t>(v) * k + pos] = nk;
    flags[static_cast<uint64_t>(v) * k + pos] = kFlagNew | kFlagReplaced;
    __hip_atomic_store(&T[vs], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (newc) newc[vs] = 1u;  // its one in-edge, flagged new
  }
}

constexpr int kRepairWaves = 16;
constexpr int kRepairHash = 2048;  // slots per table (a batch notes at most 256 ids in each)
constexpr uint32_t kTail = 4;      // list entries whose indegree a first attempt reads

template <int NR>
struct RepairShape {
  static constexpr int kSteps = NR == 1 ? 8 : 4;  // steps per wave and batch
  static constexpr int kBatch = kSteps * kRepairWaves;
};

FGIM_DEV uint32_t repair_slot(uint32_t id) { return (id * 0x9E3779B1u) >> 21; }

// A table slot packs (vertex << 32) | step; kEmptySlot is free.
constexpr uint64_t kEmptySlot = ~0ull;

// record that step i writes id (keeps the smallest step per id); returns
// the id's slot
FGIM_DEV uint32_t note_write(uint64_t* tab, uint32_t id, uint32_t i) {
  uint32_t s = repair_slot(id);
  const uint64_t mine = (static_cast<uint64_t>(id) << 32) | i;
  for (;;) {
    const uint64_t prev = atomicCAS(reinterpret_cast<unsigned long long*>(&tab[s]), kEmptySlot, mine);
    if (prev == kEmptySlot) return s;
    if (static_cast<uint32_t>(prev >> 32) == id) {
      atomicMin(reinterpret_cast<unsigned long long*>(&tab[s]), mine);
      return s;
    }
    s = (s + 1) & (kRepairHash - 1);
  }
}

// record that step i evicts id: first such step, and how many steps of the
// batch evict it
FGIM_DEV void note_evict(uint64_t* tab, uint32_t* cnt, uint32_t id, uint32_t i) {
  atomicAdd(&cnt[note_write(tab, id, i)], 1u);
}

FGIM_DEV uint32_t find_slot_chain(const uint64_t* tab, uint32_t id, uint32_t s) {
  for (;;) {
    s = (s + 1) & (kRepairHash - 1);
    const uint64_t cur = tab[s];
    if (static_cast<uint32_t>(cur >> 32) == id) return s;
    if (cur == kEmptySlot) return kNone;
  }
}

// the slot holding id (kNone: absent); one LDS read unless the home slot
// holds another vertex
FGIM_DEV uint32_t find_slot(const uint64_t* tab, uint32_t id) {
  const uint32_t s = repair_slot(id);
  const uint64_t cur = tab[s];
  if (static_cast<uint32_t>(cur >> 32) == id) return s;
  if (cur == kEmptySlot) return kNone;
  return find_slot_chain(tab, id, s);
}

// first step of the batch that writes id (kNone: none)
FGIM_DEV uint32_t first_write(const uint64_t* tab, uint32_t id) {
  const uint32_t s = find_slot(tab, id);
  return s == kNone ? kNone : static_cast<uint32_t>(tab[s]);
}

// Whether step i's reading t of id's indegree may differ from the sequential
// state: a step before i evicts id, and the batch's evictions of id (all of
// them, a bound on those before i) could bring it to 1 or below, which
// flips the test "indegree > 1".  Evictions that leave it above 1 change no
// decision, and commits lower indegrees by atomic decrements.
FGIM_DEV bool evict_conflict(const uint64_t* tab, const uint32_t* cnt, uint32_t id, uint32_t t, uint32_t i) {
  const uint32_t s = find_slot(tab, id);
  if (s == kNone) return false;
  return static_cast<uint32_t>(tab[s]) < i && t <= cnt[s] + 1u;
}

template <int NR>
__global__ void __launch_bounds__(64 * kRepairWaves) repair_kernel(uint64_t* keys, uint32_t* flags, uint32_t* T,
                                                                   uint32_t* newc, const uint32_t* zero,
                                                                   const uint64_t* zkey, const uint32_t* zcount,
                                                                   uint32_t k, uint32_t* nrep) {
  // nrep[0]: vertices repaired, nrep[3]: batches, nrep[4]: steps run alone
  constexpr int S = RepairShape<NR>::kSteps;
  constexpr uint32_t B = RepairShape<NR>::kBatch;
  __shared__ uint64_t h_list[kRepairHash];   // lists written
  __shared__ uint64_t h_evict[kRepairHash];  // indegrees lowered
  __shared__ uint32_t h_ecnt[kRepairHash];   // evictions per h_evict slot
  __shared__ uint32_t s_stop[2];  // first step of the batch that cannot commit
  const int w = threadIdx.x / 64;
  const int lane = lane_id();
  for (int t = threadIdx.x; t < kRepairHash; t += blockDim.x) {
    h_list[t] = kEmptySlot;
    h_evict[t] = kEmptySlot;
    h_ecnt[t] = 0u;
  }
  if (threadIdx.x < 2) s_stop[threadIdx.x] = kNone;
  __syncthreads();
  const uint32_t Z = *zcount;
  uint32_t fixed = 0, batches = 0, alone = 0;
  uint32_t parity = 0;
  // step i = s * kRepairWaves + w of a batch belongs to slot s of wave w;
  // the zero list and first keys of the next batch load during the commits
  uint32_t vs[S];
  uint64_t zk[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const uint32_t zi = s * kRepairWaves + w;
    vs[s] = zi < Z ? zero[zi] : kNone;
    zk[s] = zi < Z ? zkey[zi] : kSentinel;
  }
  for (uint32_t base = 0; base < Z; parity ^= 1u) {
    uint32_t v[S];
    uint64_t nk[S];
    bool has[S];
    Attempt<NR> at[S];
    uint32_t tv[S][NR];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const uint64_t ks = zk[s];
      has[s] = ks != kSentinel;
      v[s] = has[s] ? key_id(ks) : kNone;
      nk[s] = (ks & 0xFFFFFFFF00000000ull) | vs[s];
    }
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const uint32_t e = r * 64 + lane;
        const bool in = has[s] && e < k;
        at[s].lk[r] = in ? ld_wg64(&keys[static_cast<uint64_t>(v[s]) * k + e]) : kSentinel;
        at[s].lf[r] = in ? ld_wg32(&flags[static_cast<uint64_t>(v[s]) * k + e]) : 0u;
      }
    // indegrees of the farthest kTail entries first: the farthest entry
    // usually qualifies, and one qualifying entry among them is the answer
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const uint32_t e = r * 64 + lane;
        tv[s][r] = at[s].lk[r] != kSentinel && e + kTail >= k ? ld_wg32(&T[key_id(at[s].lk[r])]) : 0u;
      }
    uint32_t my_list = kNone, my_evict = kNone, my_step = 0;
    bool full[S];  // the step read every entry's indegree (else only the tail's)
#pragma unroll
    for (int s = 0; s < S; ++s) {
      decide_attempt<NR>(at[s], tv[s], k);
      full[s] = has[s] && !at[s].ok;
      if (full[s]) {
        // none of the tail qualifies: read every entry's indegree
#pragma unroll
        for (int r = 0; r < NR; ++r)
          tv[s][r] = at[s].lk[r] != kSentinel ? ld_wg32(&T[key_id(at[s].lk[r])]) : 0u;
        decide_attempt<NR>(at[s], tv[s], k);
      }
      if (!has[s]) at[s].ok = false;
      uint32_t ev = kNone;
#pragma unroll
      for (int r = 0; r < NR; ++r)
        if (at[s].ok && at[s].drop >= 0 && r == at[s].drop / 64) ev = key_id(readlane64(at[s].lk[r], at[s].drop % 64));
      if (lane == s) {
        my_step = s * kRepairWaves + w;
        my_list = at[s].ok ? v[s] : kNone;
        my_evict = ev;
      }
    }
    if (my_list != kNone) note_write(h_list, my_list, my_step);
    if (my_evict != kNone) note_evict(h_evict, h_ecnt, my_evict, my_step);
    __syncthreads();
    if (threadIdx.x == 0) s_stop[parity ^ 1u] = kNone;
    uint32_t my_stop = kNone;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const uint32_t i = s * kRepairWaves + w;
      bool stop = has[s] && !at[s].ok;
      if (at[s].ok && first_write(h_list, v[s]) < i) stop = true;
      // indegrees this step read: none for a free slot, else the tail's, or
      // every entry's after the fallback
      const bool reads_t = at[s].ok && at[s].drop >= 0;
      bool hit = false;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const uint32_t e = r * 64 + lane;
        if (reads_t && at[s].lk[r] != kSentinel && (full[s] || e + kTail >= k))
          hit |= evict_conflict(h_evict, h_ecnt, key_id(at[s].lk[r]), tv[s][r], i);
      }
      if (ballot(hit)) stop = true;
      if (stop && i < my_stop) my_stop = i;
    }
    if (lane == 0 && my_stop != kNone) atomicMin(&s_stop[parity], my_stop);
    __syncthreads();
    const uint32_t nb = Z - base < B ? Z - base : B;
    uint32_t pend = s_stop[parity] < nb ? s_stop[parity] : nb;
    const uint32_t next = base + (pend ? pend : 1u);
    uint32_t nvs[S];
    uint64_t nzk[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const uint32_t zi = next + s * kRepairWaves + w;
      nvs[s] = zi < Z ? zero[zi] : kNone;
      nzk[s] = zi < Z ? zkey[zi] : kSentinel;
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const uint32_t i = s * kRepairWaves + w;
      if (i < pend && at[s].ok) {
        commit_attempt<NR>(keys, flags, T, newc, at[s], v[s], vs[s], nk[s], k);
        ++fixed;
      }
    }
    ++batches;
    if (pend == 0) {
      // the batch's first step found no slot in its closest neighbour's list:
      // it tries the next neighbours alone (wave 0 owns step 0)
      ++alone;
      if (w == 0) {
        for (uint32_t t = 1; t < k; ++t) {
          const uint64_t ks = keys[static_cast<uint64_t>(vs[0]) * k + t];
          if (ks == kSentinel) break;
          const uint32_t vt = key_id(ks);
          const Attempt<NR> a1 = try_neighbour<NR>(keys, flags, T, vt, k);
          if (a1.ok) {
            commit_attempt<NR>(keys, flags, T, newc, a1, vt, vs[0], (ks & 0xFFFFFFFF00000000ull) | vs[0], k);
            ++fixed;
            break;
          }
        }
      }
      pend = 1;
    }
    for (int t = threadIdx.x; t < kRepairHash; t += blockDim.x) {
      h_list[t] = kEmptySlot;
      h_evict[t] = kEmptySlot;
      h_ecnt[t] = 0u;
    }
    __threadfence_block();
    __syncthreads();
    base = next;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      vs[s] = nvs[s];
      zk[s] = nzk[s];
    }
  }
  if (lane_id() == 0 && fixed) atomicAdd(nrep, fixed);
  if (threadIdx.x == 0) {
    atomicAdd(nrep + 3, batches);
    atomicAdd(nrep + 4, alone);
  }
}

// Algorithm 4 for lists of at most 32 entries.  Each wavefront slot holds two
// steps, one per half-wave (lanes 0-31 and 32-63, lane e of a half holding
// entry e of that step's neighbour list), so a batch covers kHalfBatch = 256
// steps with about the registers repair_kernel needs for 128.  The batch
// protocol is repair_kernel's: every step's first attempt against the state
// at the batch start, the two LDS tables of first writers, the longest
// conflict-free prefix, and a step whose first attempt fails run alone.
constexpr int kHalfSlots = 8;
constexpr uint32_t kHalfBatch = 2u * kHalfSlots * kRepairWaves;

// the attempt of each half's step from its list (lk, lf) and indegrees tv
FGIM_DEV void decide_half(uint64_t lk, uint32_t lf, uint32_t tv, uint32_t k, uint32_t hf, int& drop, bool& ok) {
  const uint32_t e = static_cast<uint32_t>(lane_id()) & 31u;
  const uint64_t lastk = shfl64(lk, static_cast<int>(hf * 32 + k - 1));
  const bool cand = e < k && !(lf & kFlagReplaced) && tv > 1u;
  const uint32_t hm = static_cast<uint32_t>(ballot(cand) >> (32 * hf));
  drop = -1;
  ok = true;
  if (lastk != kSentinel) {
    drop = hm ? 31 - __clz(static_cast<int>(hm)) : -1;
    ok = drop >= 0;
  }
}

__global__ void __launch_bounds__(64 * kRepairWaves) repair_half_kernel(uint64_t* keys, uint32_t* flags, uint32_t* T,
                                                                        uint32_t* newc, const uint32_t* zero,
                                                                        const uint64_t* zkey, const uint32_t* zcount,
                                                                        uint32_t k, uint32_t* nrep) {
  constexpr int S = kHalfSlots;
  constexpr uint32_t B = kHalfBatch;
  __shared__ uint64_t h_list[kRepairHash];   // lists written
  __shared__ uint64_t h_evict[kRepairHash];  // indegrees lowered
  __shared__ uint32_t h_ecnt[kRepairHash];   // evictions per h_evict slot
  __shared__ uint32_t s_stop[2];
  const uint32_t w = threadIdx.x / 64;
  const int lane = lane_id();
  const uint32_t hf = static_cast<uint32_t>(lane) >> 5;  // half
  const uint32_t e = static_cast<uint32_t>(lane) & 31u;  // list entry of the half's step
  const uint64_t hmask = hf ? 0xFFFFFFFF00000000ull : 0x00000000FFFFFFFFull;
  for (int t = threadIdx.x; t < kRepairHash; t += blockDim.x) {
    h_list[t] = kEmptySlot;
    h_evict[t] = kEmptySlot;
    h_ecnt[t] = 0u;
  }
  if (threadIdx.x < 2) s_stop[threadIdx.x] = kNone;
  __syncthreads();
  const uint32_t Z = *zcount;
  uint32_t fixed = 0, batches = 0, alone = 0;
  uint32_t parity = 0;
  // step (2s + hf) * kRepairWaves + w of a batch: slot s, half hf, wave w
  for (uint32_t base = 0; base < Z; parity ^= 1u) {
    uint32_t vs[S], v[S], lf[S], tv[S];
    uint64_t zk[S], nk[S], lk[S];
    bool has[S], ok[S], full[S];
    int drop[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const uint32_t zi = base + (2u * s + hf) * kRepairWaves + w;
      vs[s] = zi < Z ? zero[zi] : kNone;
      zk[s] = zi < Z ? zkey[zi] : kSentinel;
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
      has[s] = zk[s] != kSentinel;
      v[s] = has[s] ? key_id(zk[s]) : kNone;
      nk[s] = (zk[s] & 0xFFFFFFFF00000000ull) | vs[s];
    }
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const bool in = has[s] && e < k;
      lk[s] = in ? ld_wg64(&keys[static_cast<uint64_t>(v[s]) * k + e]) : kSentinel;
      lf[s] = in ? ld_wg32(&flags[static_cast<uint64_t>(v[s]) * k + e]) : 0u;
    }
#pragma unroll
    for (int s = 0; s < S; ++s)
      tv[s] = lk[s] != kSentinel && e + kTail >= k ? ld_wg32(&T[key_id(lk[s])]) : 0u;
    uint32_t my_list = kNone, my_evict = kNone, my_step = 0;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      decide_half(lk[s], lf[s], tv[s], k, hf, drop[s], ok[s]);
      full[s] = has[s] && !ok[s];
      if (ballot(full[s])) {
        // a half whose tail has no qualifying entry reads every indegree
        if (full[s] && lk[s] != kSentinel) tv[s] = ld_wg32(&T[key_id(lk[s])]);
        decide_half(lk[s], lf[s], tv[s], k, hf, drop[s], ok[s]);
      }
      if (!has[s]) ok[s] = false;
      const int dl = static_cast<int>(hf * 32) + (drop[s] >= 0 ? drop[s] : 0);
      const uint32_t ev = ok[s] && drop[s] >= 0 ? key_id(shfl64(lk[s], dl)) : kNone;
      // lanes 2s+h note step (s, h)'s list, lanes 32+2s+h its evicted entry
#pragma unroll
      for (uint32_t h = 0; h < 2; ++h) {
        const uint32_t vh = readlane(ok[s] ? v[s] : kNone, static_cast<int>(32 * h));
        const uint32_t eh = readlane(ev, static_cast<int>(32 * h));
        const uint32_t ih = (2u * s + h) * kRepairWaves + w;
        if (static_cast<uint32_t>(lane) == 2u * s + h) {
          my_list = vh;
          my_step = ih;
        }
        if (static_cast<uint32_t>(lane) == 32u + 2u * s + h) {
          my_evict = eh;
          my_step = ih;
        }
      }
    }
    if (my_list != kNone) note_write(h_list, my_list, my_step);
    if (my_evict != kNone) note_evict(h_evict, h_ecnt, my_evict, my_step);
    __syncthreads();
    if (threadIdx.x == 0) s_stop[parity ^ 1u] = kNone;
    uint32_t my_stop = kNone;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const uint32_t i = (2u * s + hf) * kRepairWaves + w;
      bool stop = has[s] && !ok[s];
      if (ok[s] && first_write(h_list, v[s]) < i) stop = true;
      const bool reads_t = ok[s] && drop[s] >= 0;
      const bool hit = reads_t && lk[s] != kSentinel && (full[s] || e + kTail >= k) &&
                       evict_conflict(h_evict, h_ecnt, key_id(lk[s]), tv[s], i);
      if (ballot(hit) & hmask) stop = true;
      if (stop && i < my_stop) my_stop = i;
    }
#pragma unroll
    for (int st = 32; st >= 1; st /= 2) {
      const uint32_t o = static_cast<uint32_t>(__shfl_xor(static_cast<int>(my_stop), st, 64));
      my_stop = o < my_stop ? o : my_stop;
    }
    if (lane == 0 && my_stop != kNone) atomicMin(&s_stop[parity], my_stop);
    __syncthreads();
    const uint32_t nb = Z - base < B ? Z - base : B;
    uint32_t pend = s_stop[parity] < nb ? s_stop[parity] : nb;
    // commit both halves' steps of each slot at once
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const uint32_t i = (2u * s + hf) * kRepairWaves + w;
      const bool commit = i < pend && ok[s];
      if (!ballot(commit)) continue;
      const int d = drop[s];
      const uint32_t pos = static_cast<uint32_t>(
          popc64(ballot(e < k && static_cast<int>(e) != d && lk[s] < nk[s]) & hmask));
      const int dl = static_cast<int>(hf * 32) + (d >= 0 ? d : 0);
      const uint64_t dk = shfl64(lk[s], dl);
      const uint32_t df = static_cast<uint32_t>(__shfl(static_cast<int>(lf[s]), dl, 64));
      const uint64_t row = static_cast<uint64_t>(v[s]) * k;
      if (commit && d >= 0 && e == 0) {
        __hip_atomic_fetch_sub(&T[key_id(dk)], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (newc && (df & kFlagNew)) atomicSub(&newc[key_id(dk)], 1u);
      }
      if (commit && e < k && static_cast<int>(e) != d && lk[s] != kSentinel) {
        uint32_t ne = e - (d >= 0 && static_cast<int>(e) > d ? 1u : 0u);
        if (ne >= pos) ++ne;
        if (ne < k) {
          keys[row + ne] = lk[s];
          flags[row + ne] = lf[s];
        }
      }
      if (commit && e == 0) {
        keys[row + pos] = nk[s];
        flags[row + pos] = kFlagNew | kFlagReplaced;
        __hip_atomic_store(&T[vs[s]], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        if (newc) newc[vs[s]] = 1u;
        ++fixed;
      }
    }
    ++batches;
    if (pend == 0) {
      // the batch's first step (slot 0, half 0 of wave 0) found no slot in
      // its closest neighbour's list: it tries the next neighbours alone
      ++alone;
      if (w == 0) {
        const uint32_t v0 = readlane(vs[0], 0);
        for (uint32_t t = 1; t < k; ++t) {
          const uint64_t ks = keys[static_cast<uint64_t>(v0) * k + t];
          if (ks == kSentinel) break;
          const uint32_t vt = key_id(ks);
          const Attempt<1> a1 = try_neighbour<1>(keys, flags, T, vt, k);
          if (a1.ok) {
            commit_attempt<1>(keys, flags, T, newc, a1, vt, v0, (ks & 0xFFFFFFFF00000000ull) | v0, k);
            if (lane == 0) ++fixed;
            break;
          }
        }
      }
      pend = 1;
    }
    for (int t = threadIdx.x; t < kRepairHash; t += blockDim.x) {
      h_list[t] = kEmptySlot;
      h_evict[t] = kEmptySlot;
      h_ecnt[t] = 0u;
    }
    __threadfence_block();
    __syncthreads();
    base += pend;
  }
  if (e == 0 && fixed) atomicAdd(nrep, fixed);
  if (threadIdx.x == 0) {
    atomicAdd(nrep + 3, batches);
    atomicAdd(nrep + 4, alone);
  }
}

// ---------------------------------------------------------------------------
// host driver

struct RefineBufs {
  uint64_t* keys;
  uint32_t* flags;
  uint32_t* rev_cnt;
  uint32_t* rev_off;
  uint32_t* rev_cur;
  uint64_t* rev;
  uint32_t* ptgt;
  uint64_t* pkey;   // appended proposals; the second move pass of a grouping reuses ptgt / pkey
  uint32_t* poff;
  uint32_t* bmat;   // grouping: bucket-major count matrices and their scans
  uint32_t* bmoff;
  uint32_t* bmat2;
  uint32_t* bmoff2;
  uint32_t* cseg;   // grouping: records after the first move pass
  uint64_t* cval;   // ... and, once the proposals are grouped, their keys by target
  uint32_t* T;
  uint32_t* zmask;
  uint32_t* zoff;
  uint32_t* zero;
  uint64_t* zkey;
  uint32_t* newc;  // per vertex: in-edges flagged new (nullable outside refinement)
  uint32_t* hdr;  // [0] proposals this round, [1] max per round, [2] repaired, [3] sum,
                  // [4] rechecked, [5] repair batches, [6] run alone, [16..17] pairs
                  // this round and [18..19] their largest count (64-bit)
  uint32_t* scan_tmp;
  uint64_t* sub_off;
};

static uint32_t grid_for(uint64_t n, uint32_t per_block = 256) {
  const uint64_t b = (n + per_block - 1) / per_block;
  return static_cast<uint32_t>(std::min<uint64_t>(std::max<uint64_t>(b, 1), 65536));
}

hipError_t launch_join(const JoinArgs& ja, int nr, int mmax, uint32_t grid, size_t smem, hipStream_t s) {
#define FGIM_JOIN_CASE(NR_, MM_)                                                               \
  if (nr == NR_ && mmax == MM_) {                                                              \
    hipLaunchKernelGGL((join_kernel<NR_, MM_>), dim3(grid), dim3(256), smem, s, ja);           \
    return hipGetLastError();                                                                  \
  }
  FGIM_JOIN_CASE(1, 4)
  FGIM_JOIN_CASE(2, 4)
  FGIM_JOIN_CASE(1, 16)
  FGIM_JOIN_CASE(2, 16)
#undef FGIM_JOIN_CASE
  return hipErrorInvalidValue;
}

struct RoundPlan {
  uint64_t N;
  uint32_t k, k_rev, cap;
  bool repair;
  JoinArgs ja;
  int nr, mmax;
  uint32_t join_grid, cand_grid, recheck_grid;
  size_t join_smem;
  bool use_mfma;
  BucketPlan prop_plan, rev_plan;
  uint32_t batches;  // > 1: streamlined rounds of this many vertex ranges
  uint32_t chunks;   // Update of a synchronous round in this many vertex chunks (MFMA join)
};

// indegrees T of the lists in b.keys
hipError_t launch_indegree(const RefineBufs& b, uint64_t N, uint32_t k, hipStream_t s) {
  const uint64_t nk = N * k;
  hipError_t e;
  if ((e = fill_u32(b.T, 0u, N, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(indegree_kernel, dim3(grid_for(nk)), dim3(256), 0, s, b.keys, nk, b.T);
  return hipGetLastError();
}

// Algorithm 4 on the lists in b.keys with their indegrees in b.T (kept
// current, with b.newc when set); repaired count added to b.hdr[2]
hipError_t launch_repair(const RefineBufs& b, uint64_t N, uint32_t k, hipStream_t s) {
  hipError_t e;
  hipLaunchKernelGGL(zero_mask_kernel, dim3(grid_for(N)), dim3(256), 0, s, b.T, b.keys, k, N, b.zmask);
  if ((e = exclusive_scan(b.zmask, b.zoff, N, b.scan_tmp, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(zero_compact_kernel, dim3(grid_for(N)), dim3(256), 0, s, b.zmask, b.zoff, N, b.keys, k, b.zero,
                     b.zkey);
  if (k <= 32)
    hipLaunchKernelGGL(repair_half_kernel, dim3(1), dim3(64 * kRepairWaves), 0, s, b.keys, b.flags, b.T, b.newc,
                       b.zero, b.zkey, b.zoff + N, k, b.hdr + 2);
  else if (k <= 64)
    hipLaunchKernelGGL(repair_kernel<1>, dim3(1), dim3(64 * kRepairWaves), 0, s, b.keys, b.flags, b.T, b.newc, b.zero,
                       b.zkey, b.zoff + N, k, b.hdr + 2);
  else
    hipLaunchKernelGGL(repair_kernel<2>, dim3(1), dim3(64 * kRepairWaves), 0, s, b.keys, b.flags, b.T, b.newc, b.zero,
                       b.zkey, b.zoff + N, k, b.hdr + 2);
  return hipGetLastError();
}

// one refinement round; only kernel launches (graph-capturable)
hipError_t run_stream_round(const RoundPlan& rp, const RefineBufs& b, hipStream_t s);

hipError_t run_round(const RoundPlan& rp, const RefineBufs& b, hipStream_t s) {
  if (rp.batches > 1) return run_stream_round(rp, b, s);
  const uint64_t N = rp.N, nk = N * rp.k;
  hipError_t e;
  // Visit: active vertices from the maintained new in-edge counts, then
  // the reverse CSR (b.zmask holds the active flags until the repair
  // reuses it)
  hipLaunchKernelGGL(rev_active_kernel, dim3(grid_for(N)), dim3(256), 0, s, b.newc, b.flags, rp.k, N, b.zmask);
  if ((e = fill_u32(b.newc, 0u, N, s)) != hipSuccess) return e;
  if ((e = group_records(RevRecords{b.keys, b.flags, b.zmask, nk, rp.k}, rp.rev_plan, b.bmat, b.bmoff, b.bmat2,
                         b.bmoff2, b.scan_tmp, b.cseg, b.cval, b.ptgt, b.pkey, b.rev_off, b.rev, s)) != hipSuccess)
    return e;
  // Update, in vertex chunks that share one pair buffer: every chunk joins
  // against the same snapshot, and the proposals of all of them are applied
  // together, so the chunking changes no result
  if ((e = fill_u32(b.hdr, 0u, 1, s)) != hipSuccess) return e;
  if (rp.use_mfma) {
    const uint64_t cus = static_cast<uint64_t>(device_cus());
    // the screen reads every candidate's data, later chunks' vertices too
    if (rp.chunks > 1)
      hipLaunchKernelGGL(aux_refresh_kernel, dim3(grid_for(N)), dim3(256), 0, s, b.keys, N, rp.k, rp.ja.nrm2,
                         rp.ja.qerr2, rp.ja.dim, rp.ja.aux);
    for (uint32_t c = 0; c < rp.chunks; ++c) {
      JoinArgs ja = rp.ja;
      ja.u_lo = N * c / rp.chunks;
      ja.u_hi = N * (c + 1) / rp.chunks;
      const uint64_t n = ja.u_hi - ja.u_lo;
      if (n == 0) continue;
      if ((e = fill_u32(reinterpret_cast<uint32_t*>(ja.npairs), 0u, 2, s)) != hipSuccess) return e;
      hipLaunchKernelGGL(cand_kernel, dim3(static_cast<uint32_t>(std::min<uint64_t>((n + 3) / 4, cus * 16))), dim3(256),
                         0, s, ja);
      hipLaunchKernelGGL(join_mfma_kernel, dim3(static_cast<uint32_t>(std::min<uint64_t>(n, cus * 8))), dim3(256),
                         rp.join_smem, s, ja);
      if (rp.mmax == 4)
        hipLaunchKernelGGL(recheck_kernel<4>, dim3(rp.recheck_grid), dim3(256), 0, s, ja);
      else
        hipLaunchKernelGGL(recheck_kernel<16>, dim3(rp.recheck_grid), dim3(256), 0, s, ja);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
  } else if ((e = launch_join(rp.ja, rp.nr, rp.mmax, rp.join_grid, rp.join_smem, s)) != hipSuccess) {
    return e;
  }
  // the proposals' keys end up grouped in b.cval (the append buffer serves
  // the second move pass)
  if ((e = group_records(PropRecords{b.ptgt, b.pkey, b.hdr, rp.cap}, rp.prop_plan, b.bmat, b.bmoff, b.bmat2,
                         b.bmoff2, b.scan_tmp, b.cseg, b.cval, b.ptgt, b.pkey, b.poff, b.cval, s)) != hipSuccess)
    return e;
  if (rp.nr == 1)
    hipLaunchKernelGGL(apply_kernel<1>, dim3(grid_for(N, 4)), dim3(256), 0, s, b.keys, b.flags, N, rp.k, b.poff,
                       b.cval, b.hdr + 1, b.hdr, b.T, b.newc);
  else
    hipLaunchKernelGGL(apply_kernel<2>, dim3(grid_for(N, 4)), dim3(256), 0, s, b.keys, b.flags, N, rp.k, b.poff,
                       b.cval, b.hdr + 1, b.hdr, b.T, b.newc);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (!rp.repair) return hipSuccess;
  return launch_repair(b, N, rp.k, s);
}

// A streamlined round (Section 4.2.1): the vertex ranges [t N / B,
// (t + 1) N / B) in turn, each a Visit + Update on the lists the ranges
// before it left, its proposals applied before the next range; indegree
// repair at the end, as in a synchronous round.
hipError_t run_stream_round(const RoundPlan& rp, const RefineBufs& b, hipStream_t s) {
  const uint64_t N = rp.N, nk = N * rp.k;
  const uint64_t cus = static_cast<uint64_t>(device_cus());
  hipError_t e;
  for (uint32_t t = 0; t < rp.batches; ++t) {
    const uint64_t lo = N * t / rp.batches, hi = N * (t + 1) / rp.batches;
    if (lo == hi) continue;
    JoinArgs ja = rp.ja;
    ja.u_lo = lo;
    ja.u_hi = hi;
    const uint64_t n = hi - lo;
    // Visit: reverse segments of the range's vertices only, from the
    // recorded links; then links are consumed and recorded
    if ((e = fill_u32(b.rev_cnt, 0u, 2 * N, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(rev_count_range_kernel, dim3(grid_for(nk)), dim3(256), 0, s, b.keys, b.flags, nk, rp.k, lo, hi,
                       b.rev_cnt);
    hipLaunchKernelGGL(rev_active_range_kernel, dim3(grid_for(N)), dim3(256), 0, s, b.flags, N, rp.k, lo, hi, b.rev_cnt,
                       b.zmask);
    if ((e = exclusive_scan(b.rev_cnt, b.rev_off, 2 * N, b.scan_tmp, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(copy_u32_kernel, dim3(grid_for(2 * N)), dim3(256), 0, s, b.rev_off, b.rev_cur, 2 * N);
    hipLaunchKernelGGL(rev_scatter_range_kernel, dim3(grid_for(nk)), dim3(256), 0, s, b.keys, b.flags, nk, rp.k, lo, hi,
                       b.zmask, b.rev_cur, b.rev);
    // Update of the range
    if ((e = fill_u32(b.hdr, 0u, 1, s)) != hipSuccess) return e;
    if (rp.use_mfma) {
      hipLaunchKernelGGL(aux_refresh_kernel, dim3(grid_for(N)), dim3(256), 0, s, b.keys, N, rp.k, ja.nrm2, ja.qerr2,
                         ja.dim, ja.aux);
      if ((e = fill_u32(reinterpret_cast<uint32_t*>(ja.npairs), 0u, 2, s)) != hipSuccess) return e;
      hipLaunchKernelGGL(cand_kernel, dim3(static_cast<uint32_t>(std::min<uint64_t>((n + 3) / 4, cus * 16))), dim3(256),
                         0, s, ja);
      hipLaunchKernelGGL(join_mfma_kernel, dim3(static_cast<uint32_t>(std::min<uint64_t>(n, cus * 8))), dim3(256),
                         rp.join_smem, s, ja);
      if (rp.mmax == 4)
        hipLaunchKernelGGL(recheck_kernel<4>, dim3(rp.recheck_grid), dim3(256), 0, s, ja);
      else
        hipLaunchKernelGGL(recheck_kernel<16>, dim3(rp.recheck_grid), dim3(256), 0, s, ja);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    } else if ((e = launch_join(ja, rp.nr, rp.mmax, static_cast<uint32_t>(std::min<uint64_t>(n, cus * 8)), rp.join_smem,
                                s)) != hipSuccess) {
      return e;
    }
    if ((e = group_records(PropRecords{b.ptgt, b.pkey, b.hdr, rp.cap}, rp.prop_plan, b.bmat, b.bmoff, b.bmat2,
                           b.bmoff2, b.scan_tmp, b.cseg, b.cval, b.ptgt, b.pkey, b.poff, b.cval, s)) != hipSuccess)
      return e;
    if (rp.nr == 1)
      hipLaunchKernelGGL(apply_stream_kernel<1>, dim3(grid_for(N, 4)), dim3(256), 0, s, b.keys, b.flags, N, rp.k, lo, hi,
                         b.poff, b.cval, b.hdr + 1, b.hdr, b.T);
    else
      hipLaunchKernelGGL(apply_stream_kernel<2>, dim3(grid_for(N, 4)), dim3(256), 0, s, b.keys, b.flags, N, rp.k, lo, hi,
                         b.poff, b.cval, b.hdr + 1, b.hdr, b.T);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (!rp.repair) return hipSuccess;
  return launch_repair(b, N, rp.k, s);
}

uint32_t ceil_pow2_u(uint32_t x) {
  uint32_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

__global__ void check_ids_kernel(const uint32_t* ids, uint64_t nk, uint64_t N, uint32_t* err) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < nk;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    if (ids[i] != kNone && ids[i] >= N) atomicOr(err, 1u);
}

// largest proposals and screened pairs per vertex that a refinement round
// has needed in this process (sizes the buffers of later calls)
std::mutex g_demand_mu;
double g_props_per_vertex = 0.0, g_pairs_per_vertex = 0.0;

// Stage 2 on the lists (ids, dist).  Lists from a caller are checked first
// (an id >= n would index the indegrees out of bounds); the merge passes its
// own stage-1 lists as trusted and skips the check and its host wait.
fgim_status refine_impl(const fgim_dataset* d, const fgim_params* p, uint32_t* ids, float* dist, uint32_t* T_out,
                        fgim_stats* stats, hipStream_t s, bool trusted) {
  FGIM_TRY(check_dataset(d, false));
  if (!p) return fail(FGIM_ERR_INVALID_ARG, "params is NULL");
  if (!ids || !dist) return fail(FGIM_ERR_INVALID_ARG, "lists are NULL");
  if (p->k == 0 || p->k > FGIM_MAX_K) return fail(FGIM_ERR_INVALID_ARG, "k = %u out of 1..%u", p->k, FGIM_MAX_K);
  const uint32_t k_rev = p->k_rev ? p->k_rev : p->k;
  if (k_rev > FGIM_MAX_K) return fail(FGIM_ERR_INVALID_ARG, "k_rev = %u > %u", k_rev, FGIM_MAX_K);
  const uint64_t N = d->n_total, nk = N * p->k;
  if (nk >= 0xFFFFFFFFull || 2 * N + 1 >= 0xFFFFFFFFull)
    return fail(FGIM_ERR_UNSUPPORTED, "N x k = %llu list entries exceed 32-bit offsets", (unsigned long long)nk);
  const bool repair = !(p->flags & FGIM_FLAG_NO_REPAIR);
  if (p->stream_batches > FGIM_MAX_STREAM_BATCHES)
    return fail(FGIM_ERR_INVALID_ARG, "stream_batches = %u > %u", p->stream_batches, FGIM_MAX_STREAM_BATCHES);
  if (p->update_chunks > FGIM_MAX_STREAM_BATCHES)
    return fail(FGIM_ERR_INVALID_ARG, "update_chunks = %u > %u", p->update_chunks, FGIM_MAX_STREAM_BATCHES);
  if (!trusted) {
    Scratch chk(s);
    uint32_t* err = nullptr;
    FGIM_TRY(chk.get(&err, 4));
    HIP_TRY(fill_u32(err, 0u, 1, s));
    hipLaunchKernelGGL(check_ids_kernel, dim3(grid_for(nk)), dim3(256), 0, s, ids, nk, N, err);
    HIP_TRY(hipGetLastError());
    uint32_t herr = 0;
    HIP_TRY(hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (herr) return fail(FGIM_ERR_GRAPH, "a k-NN list holds an id >= n_total");
  }

  const uint32_t dim = d->dim, nc = dim / 4;
  const uint32_t Nch = ceil_pow2_u(nc);
  const uint32_t P = std::min<uint32_t>(64, std::max<uint32_t>(std::min<uint32_t>(4, Nch), Nch / 4));
  const uint32_t M = Nch / P;
  const uint32_t ccap = 2 * (p->k + k_rev);
  const size_t base_smem = static_cast<size_t>(ccap) * (4 * 4 + 8) + 8 * 4 + kPropStage * 12;
  const size_t rows_smem = static_cast<size_t>(ccap) * (dim + 4) * 4;
  const bool stage_rows = base_smem + rows_smem <= 96 * 1024;

  // MFMA join when the candidate set fits its tile layout (|Cn| + |Co| <= 128)
  const bool use_mfma = ccap <= kMfmaMaxC && !(p->flags & FGIM_FLAG_NO_MFMA_SCREEN);
  const uint32_t dpad = (dim + 31) / 32 * 32;
  const uint32_t slice = std::min<uint32_t>(dpad, 128);
  const size_t mfma_head = kMfmaMaxC * (8 + 4 * 4) + 2 * kMfmaMaxCn * 8 + 68 * 4 + 16 * 4;
  // BF16 slices of the candidate rows in LDS (FP32 rows there cost occupancy
  // and measured slower); the exact re-scoring reads FP32 rows from memory
  const size_t mfma_smem = mfma_head + static_cast<size_t>(kMfmaMaxC) * (slice + 8) * 2;

  uint64_t cap = std::max<uint64_t>(N * std::max<uint32_t>(4 * p->k, 64), 1 << 16);
  // Pairs passing the screen: about k per vertex in the first round at
  // k = 32 on clustered data, several times that on others.  The pair
  // buffer holds one chunk of the Update's vertices at a time and is kept
  // within kPairBudget; the chunk count follows from the expected demand
  // (the per-vertex demand seen so far in this process, else 3k).  A chunk
  // that overflows re-runs the rounds with a larger buffer, or, at the
  // budget, with more chunks.
  const uint64_t reserve = static_cast<uint64_t>(device_cus()) * 8 * kPairChunk;
  double ppv = 3.0 * p->k;
  {
    std::lock_guard<std::mutex> lock(g_demand_mu);
    cap = std::max<uint64_t>(cap, static_cast<uint64_t>(g_props_per_vertex * 1.25 * static_cast<double>(N)) + 1024);
    if (g_pairs_per_vertex > 0.0) ppv = g_pairs_per_vertex;
  }
  // The unit of one Update pass: a streamlined micro-batch, or a chunk of a
  // synchronous round (whose count may grow on overflow).
  const bool streamed = p->stream_batches > 1;
  const uint64_t pair_limit = streamed ? 0xF0000000ull : kPairBudget;
  uint32_t chunks = streamed ? 1u : p->update_chunks;
  if (chunks == 0) {
    const double demand = ppv * 1.25 * static_cast<double>(N);
    chunks = static_cast<uint32_t>(std::min<double>(std::ceil(demand / static_cast<double>(kPairBudget - reserve)), N));
    chunks = std::max<uint32_t>(chunks, 1);
  }
  auto unit_len = [&]() -> uint64_t {
    const uint64_t parts = streamed ? p->stream_batches : chunks;
    return std::min<uint64_t>(N, (N + parts - 1) / parts + 1);
  };
  uint64_t pair_cap = std::min<uint64_t>(static_cast<uint64_t>(ppv * 1.25 * static_cast<double>(unit_len())) + reserve,
                                         pair_limit);
  pair_cap = std::max<uint64_t>(pair_cap, 1 << 16);
  if (p->flags & FGIM_FLAG_MIN_BUFFERS) {
    cap = 1 << 16;
    pair_cap = 1 << 16;
  }
  cap = std::min<uint64_t>(cap, 0xF0000000ull);

  for (int attempt = 0; attempt < 4; ++attempt) {
    Scratch scr(s);
    RefineBufs b{};
    FGIM_TRY(scr.get(&b.keys, nk));
    FGIM_TRY(scr.get(&b.flags, nk));
    FGIM_TRY(scr.get(&b.rev_cnt, 2 * N + 1));
    FGIM_TRY(scr.get(&b.rev_off, 2 * N + 1));
    FGIM_TRY(scr.get(&b.rev_cur, 2 * N + 1));
    FGIM_TRY(scr.get(&b.rev, nk));
    // the append buffer also serves the grouping of the reverse entries
    FGIM_TRY(scr.get(&b.ptgt, std::max<uint64_t>(cap, nk)));
    FGIM_TRY(scr.get(&b.pkey, std::max<uint64_t>(cap, nk)));
    FGIM_TRY(scr.get(&b.poff, N + 1));
    const BucketPlan prop_plan = bucket_plan(N, cap), rev_plan = bucket_plan(2 * N, nk);
    const uint64_t mat_words = std::max(prop_plan.words1(), rev_plan.words1());
    const uint64_t mat2_words = std::max(prop_plan.words2(), rev_plan.words2());
    FGIM_TRY(scr.get(&b.bmat, mat_words));
    FGIM_TRY(scr.get(&b.bmoff, mat_words + 1));
    FGIM_TRY(scr.get(&b.bmat2, mat2_words));
    FGIM_TRY(scr.get(&b.bmoff2, mat2_words + 1));
    FGIM_TRY(scr.get(&b.cseg, std::max<uint64_t>(cap, nk)));
    FGIM_TRY(scr.get(&b.cval, std::max<uint64_t>(cap, nk)));
    FGIM_TRY(scr.get(&b.T, N));
    FGIM_TRY(scr.get(&b.newc, N));
    FGIM_TRY(scr.get(&b.zmask, N + 1));
    FGIM_TRY(scr.get(&b.zoff, N + 1));
    FGIM_TRY(scr.get(&b.zero, N + 1));
    FGIM_TRY(scr.get(&b.zkey, N + 1));
    FGIM_TRY(scr.get(&b.hdr, 24));
    float *nrm2 = nullptr, *qerr2 = nullptr;
    uint32_t *cand = nullptr, *ccnt = nullptr;
    uint16_t* xb = nullptr;
    uint64_t* pairs = nullptr;
    CandAux* aux = nullptr;
    if (use_mfma) {
      FGIM_TRY(scr.get(&nrm2, N));
      FGIM_TRY(scr.get(&qerr2, N));
      FGIM_TRY(scr.get(&cand, unit_len() * kMfmaMaxC));
      FGIM_TRY(scr.get(&ccnt, 2 * unit_len()));
      FGIM_TRY(scr.get(&aux, N));
      FGIM_TRY(scr.get(&pairs, pair_cap));
      // the screen's error bound is derived for round-to-nearest-even BF16
      // operands, so the join stages its own copy (never a caller's)
      if (dim % 8 == 0) {
        FGIM_TRY(scr.get(&xb, N * dim));
        FGIM_TRY(quantize_into(d->base, N, dim, d->ld, FGIM_BF16, xb, nullptr, s));
      }
      hipLaunchKernelGGL(row_norms_kernel, dim3(grid_for(N, 4)), dim3(256), 0, s, d->base, N, dim, d->ld, nrm2, qerr2);
      HIP_TRY(hipGetLastError());
    }
    FGIM_TRY(scr.get(&b.scan_tmp,
                     scan_tmp_words(std::max(std::max<uint64_t>(2 * N + 1, mat_words), mat2_words)) + 16));
    FGIM_TRY(scr.get(&b.sub_off, d->h));
    std::vector<uint64_t> hoff(d->h);
    for (uint32_t i = 0; i < d->h; ++i) hoff[i] = d->subs[i].row_offset;
    HIP_TRY(hipMemcpyAsync(b.sub_off, hoff.data(), 8 * d->h, hipMemcpyHostToDevice, s));
    HIP_TRY(fill_u32(b.hdr, 0u, 24, s));
    hipLaunchKernelGGL(to_keys_kernel, dim3(grid_for(nk)), dim3(256), 0, s, ids, dist, nk, b.keys, b.flags);
    HIP_TRY(hipGetLastError());
    // indegrees of the input lists, all of whose entries are new; apply and
    // repair keep both counts current from here on
    HIP_TRY(launch_indegree(b, N, p->k, s));
    HIP_TRY(hipMemcpyAsync(b.newc, b.T, 4 * N, hipMemcpyDeviceToDevice, s));

    RoundPlan rp{};
    rp.N = N;
    rp.k = p->k;
    rp.k_rev = k_rev;
    rp.cap = static_cast<uint32_t>(cap);
    rp.repair = repair;
    rp.nr = std::max(p->k, k_rev) <= 64 ? 1 : 2;
    rp.mmax = M <= 4 ? 4 : 16;
    rp.batches = p->stream_batches;
    rp.chunks = chunks;
    JoinArgs& ja = rp.ja;
    ja.X = d->base;
    ja.ld = d->ld;
    ja.nc = nc;
    ja.metric = d->metric;
    ja.N = N;
    ja.k = p->k;
    ja.k_rev = k_rev;
    ja.keys = b.keys;
    ja.flags = b.flags;
    ja.rev_off = b.rev_off;
    ja.rev = b.rev;
    ja.sub_off = b.sub_off;
    ja.h = d->h;
    ja.cap = rp.cap;
    ja.ptotal = b.hdr;
    ja.ptgt = b.ptgt;
    ja.pkey = b.pkey;
    ja.P = P;
    ja.M = M;
    ja.ccap = ccap;
    ja.stage_rows = stage_rows;
    ja.nrm2 = nrm2;
    ja.qerr2 = qerr2;
    ja.xb = xb;
    ja.dim = dim;
    ja.dpad = dpad;
    ja.slice = slice;
    ja.rechecked = b.hdr + 4;
    ja.cand = cand;
    ja.ccnt = ccnt;
    ja.aux = aux;
    ja.pairs = pairs;
    ja.npairs = reinterpret_cast<unsigned long long*>(b.hdr + 16);
    ja.npairs_max = reinterpret_cast<unsigned long long*>(b.hdr + 18);
    ja.pair_cap = static_cast<uint32_t>(pair_cap);
    ja.u_lo = 0;
    ja.u_hi = N;
    rp.use_mfma = use_mfma;
    rp.prop_plan = prop_plan;
    rp.rev_plan = rev_plan;
    rp.join_smem = use_mfma ? mfma_smem : base_smem + (stage_rows ? rows_smem : 0);
    rp.join_grid = static_cast<uint32_t>(std::min<uint64_t>(N, static_cast<uint64_t>(device_cus()) * 8));
    rp.cand_grid = static_cast<uint32_t>(std::min<uint64_t>((N + 3) / 4, static_cast<uint64_t>(device_cus()) * 16));
    rp.recheck_grid = static_cast<uint32_t>(device_cus()) * 8;
    if (use_mfma && rp.join_smem > 64 * 1024)
      HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(join_mfma_kernel),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(rp.join_smem)));
    if (!use_mfma && rp.join_smem > 64 * 1024)
      HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(rp.nr == 1 ? (rp.mmax == 4 ? join_kernel<1, 4> : join_kernel<1, 16>)
                                                                           : (rp.mmax == 4 ? join_kernel<2, 4> : join_kernel<2, 16>)),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(rp.join_smem)));

    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (stats) {
      HIP_TRY(hipEventCreate(&e0));
      HIP_TRY(hipEventCreate(&e1));
      HIP_TRY(hipEventRecord(e0, s));
    }
    const bool capture = !(p->flags & FGIM_FLAG_NO_GRAPH_CAPTURE) && p->rounds > 1;
    if (capture) {
      // The first round runs directly on the caller's stream; while the
      // device works on it, the host captures one round into a graph and
      // instantiates it, and the remaining rounds replay that graph.
      // Capture needs a stream other than the legacy null stream, so the
      // replays run on a library stream ordered after, and before, the
      // caller's stream by events.
      HIP_TRY(run_round(rp, b, s));
      hipStream_t cs = nullptr;
      HIP_TRY(library_stream(&cs));
      hipEvent_t joined = nullptr, done = nullptr;
      HIP_TRY(hipEventCreateWithFlags(&joined, hipEventDisableTiming));
      HIP_TRY(hipEventCreateWithFlags(&done, hipEventDisableTiming));
      HIP_TRY(hipEventRecord(joined, s));
      HIP_TRY(hipStreamWaitEvent(cs, joined, 0));
      hipGraph_t graph = nullptr;
      hipGraphExec_t exec = nullptr;
      HIP_TRY(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
      hipError_t le = run_round(rp, b, cs);
      hipError_t ce = hipStreamEndCapture(cs, &graph);
      hipError_t ie = hipSuccess;
      if (le == hipSuccess && ce == hipSuccess) ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      hipError_t ge = hipSuccess;
      for (uint32_t r = 1; r < p->rounds && le == hipSuccess && ce == hipSuccess && ie == hipSuccess && ge == hipSuccess; ++r)
        ge = hipGraphLaunch(exec, cs);
      HIP_TRY(hipEventRecord(done, cs));
      HIP_TRY(hipStreamWaitEvent(s, done, 0));
      HIP_TRY(hipStreamSynchronize(cs));
      if (exec) (void)hipGraphExecDestroy(exec);
      if (graph) (void)hipGraphDestroy(graph);
      (void)hipEventDestroy(joined);
      (void)hipEventDestroy(done);
      hipError_t first = le != hipSuccess ? le : (ce != hipSuccess ? ce : (ie != hipSuccess ? ie : ge));
      if (first != hipSuccess) return fail(FGIM_ERR_DEVICE, "refinement graph failed: %s", hipGetErrorString(first));
    } else {
      for (uint32_t r = 0; r < p->rounds; ++r) HIP_TRY(run_round(rp, b, s));
    }
    uint32_t hh[24] = {};
    HIP_TRY(hipMemcpyAsync(hh, b.hdr, sizeof(hh), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const uint64_t pairs_max = static_cast<uint64_t>(hh[18]) | (static_cast<uint64_t>(hh[19]) << 32);
    {
      std::lock_guard<std::mutex> lock(g_demand_mu);
      g_props_per_vertex = std::max(g_props_per_vertex, static_cast<double>(hh[1]) / static_cast<double>(N));
      // the pair demand is the largest Update unit's, per vertex of a unit
      const uint64_t parts = streamed ? p->stream_batches : chunks;
      const double unit_n = static_cast<double>((N + parts - 1) / parts);
      g_pairs_per_vertex = std::max(g_pairs_per_vertex, static_cast<double>(pairs_max) / unit_n);
    }
    if (hh[1] > cap || pairs_max > pair_cap) {
      // a buffer overflowed: run again with larger ones (same result)
      // later rounds of a truncated run may have needed less than a full
      // run does: at least double the buffer that overflowed
      if (hh[1] > cap) cap = std::min<uint64_t>(std::max<uint64_t>(static_cast<uint64_t>(hh[1]) * 5 / 4, 2 * cap) + 1024, 0xF0000000ull);
      if (pairs_max > pair_cap) {
        const uint64_t want = std::max<uint64_t>(pairs_max * 5 / 4, 2 * pair_cap) + 1024;
        if (want <= pair_limit) {
          pair_cap = want;
        } else if (streamed) {
          pair_cap = pair_limit;
        } else {
          // at the budget: split the Update into proportionally more chunks
          pair_cap = kPairBudget;
          const double grow = std::ceil(static_cast<double>(pairs_max) * 1.25 / static_cast<double>(kPairBudget - reserve));
          chunks = static_cast<uint32_t>(std::min<double>(static_cast<double>(chunks) * std::max(2.0, grow), N));
        }
      }
      continue;
    }
    hipLaunchKernelGGL(from_keys_kernel, dim3(grid_for(nk)), dim3(256), 0, s, b.keys, nk, ids, dist);
    HIP_TRY(hipGetLastError());
    if (T_out) HIP_TRY(hipMemcpyAsync(T_out, b.T, 4 * N, hipMemcpyDeviceToDevice, s));
    if (stats) {
      HIP_TRY(hipEventRecord(e1, s));
      HIP_TRY(hipEventSynchronize(e1));
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
      stats->ms_stage[1] = ms;
      stats->repaired = hh[2];
      stats->proposals = hh[3];
      stats->rechecked = hh[4];
      stats->repair_batches = hh[5];
      stats->repair_alone = hh[6];
      stats->refine_attempts = static_cast<uint32_t>(attempt + 1);
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
    }
    return FGIM_OK;
  }
  return fail(FGIM_ERR_OUT_OF_MEMORY, "join proposals keep overflowing the buffer");
}

fgim_status repair_impl(uint32_t* ids, float* dist, uint64_t N, uint32_t k, uint32_t* T_out, uint64_t* repaired,
                        hipStream_t s) {
  if (!ids || !dist) return fail(FGIM_ERR_INVALID_ARG, "NULL buffer");
  if (N == 0 || N >= 0xFFFFFFFFull) return fail(FGIM_ERR_INVALID_ARG, "n = %llu out of range", (unsigned long long)N);
  if (k == 0 || k > FGIM_MAX_K) return fail(FGIM_ERR_INVALID_ARG, "k = %u out of 1..%u", k, FGIM_MAX_K);
  const uint64_t nk = N * k;
  Scratch scr(s);
  RefineBufs b{};
  FGIM_TRY(scr.get(&b.keys, nk));
  FGIM_TRY(scr.get(&b.flags, nk));
  FGIM_TRY(scr.get(&b.T, N));
  FGIM_TRY(scr.get(&b.zmask, N + 1));
  FGIM_TRY(scr.get(&b.zoff, N + 1));
  FGIM_TRY(scr.get(&b.zero, N + 1));
  FGIM_TRY(scr.get(&b.zkey, N + 1));
  FGIM_TRY(scr.get(&b.scan_tmp, scan_tmp_words(N + 1) + 16));
  FGIM_TRY(scr.get(&b.hdr, 8));
  HIP_TRY(fill_u32(b.hdr, 0u, 8, s));
  // an id >= n would index T out of bounds: reject the lists first
  hipLaunchKernelGGL(check_ids_kernel, dim3(grid_for(nk)), dim3(256), 0, s, ids, nk, N, b.hdr + 1);
  HIP_TRY(hipGetLastError());
  uint32_t herr = 0;
  HIP_TRY(hipMemcpyAsync(&herr, b.hdr + 1, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (herr) return fail(FGIM_ERR_GRAPH, "a k-NN list holds an id >= n");
  hipLaunchKernelGGL(to_keys_kernel, dim3(grid_for(nk)), dim3(256), 0, s, ids, dist, nk, b.keys, b.flags);
  HIP_TRY(hipGetLastError());
  HIP_TRY(launch_indegree(b, N, k, s));
  HIP_TRY(launch_repair(b, N, k, s));
  hipLaunchKernelGGL(from_keys_kernel, dim3(grid_for(nk)), dim3(256), 0, s, b.keys, nk, ids, dist);
  HIP_TRY(hipGetLastError());
  if (T_out) HIP_TRY(hipMemcpyAsync(T_out, b.T, 4 * N, hipMemcpyDeviceToDevice, s));
  if (repaired) {
    uint32_t hh[4] = {0, 0, 0, 0};
    HIP_TRY(hipMemcpyAsync(hh, b.hdr, sizeof(hh), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *repaired = hh[2];
  }
  return FGIM_OK;
}

}  // namespace fgim

extern "C" fgim_status fgim_repair(uint32_t* knn_ids, float* knn_dist, uint64_t n, uint32_t k, uint32_t* indegree,
                                   uint64_t* repaired, void* stream) {
  fgim::fail(FGIM_OK, "");
  return fgim::repair_impl(knn_ids, knn_dist, n, k, indegree, repaired, static_cast<hipStream_t>(stream));
}

extern "C" fgim_status fgim_refine(const fgim_dataset* data, const fgim_params* params, uint32_t* knn_ids,
                                   float* knn_dist, uint32_t* indegree, fgim_stats* stats, void* stream) {
  fgim::fail(FGIM_OK, "");
  if (stats) memset(stats, 0, sizeof(*stats));
  return fgim::refine_impl(data, params, knn_ids, knn_dist, indegree, stats, static_cast<hipStream_t>(stream), false);
}
