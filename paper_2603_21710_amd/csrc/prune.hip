// Stage 3 of FGIM: k-NNG -> PG (Section 4.3, Algorithm 5), and the
// three-stage merge entry point.
//
//   select   per vertex u: the k x k occlusion tile of u's list (whether
//            delta(w, v) <= delta(u, v) for every earlier entry w), then the
//            sequential scan of Algorithm 5 over 64-bit masks: v is kept
//            when T(v) = 1 or no kept w occludes it; at most R are kept.
//            For k <= 64 one wavefront per vertex screens the tile on MFMA
//            (BF16 rows in LDS, rigorous error bound) and re-scores only the
//            undecided pairs in canonical FP32; otherwise one workgroup per
//            vertex scores every pair in FP32 from rows staged in LDS.
//   reverse  CSR of the selected edges by head (count / scan / scatter).
//   fill     per vertex: first R of its selected neighbours and the vertices
//            that selected it, (delta, id)-sorted and id-unique.
#include <string.h>

#include "fgim_internal.h"
#include "graph_util.h"
#include "host_util.h"
#include "mfma_util.h"

namespace fgim {

struct SelectArgs {
  const float* X;
  uint64_t ld;
  uint32_t nc;
  int metric;
  uint64_t N;
  uint32_t k, R;
  const uint32_t* ids;
  const float* dist;
  const uint32_t* T;
  uint32_t* sel_ids;   // N x R
  float* sel_dist;
  uint32_t* sel_n;
  uint32_t P, M;
  int stage_rows;
  // MFMA screen
  const float* nrm2;   // squared FP32 norm of every row
  const float* qerr2;  // squared norm of every row's BF16 rounding residual
  uint32_t dpad;       // dim rounded up to 32
  uint32_t wave_smem;  // LDS bytes per wavefront
  // selection rule (FGIM_SELECT_*) and its FP32 constants: alpha^2 or 3 tau
  uint32_t rule;
  float a2, t3;
};

// The Euclidean distance behind delta: sqrt(delta) for squared L2 and
// sqrt(2 delta) for cosine on unit vectors, a negative rounding residue read
// as 0.  The square root is correctly rounded (HIP's default for sqrtf).
FGIM_DEV float euclid_of(float d, int metric) {
  const float s = metric == kCos ? 2.0f * d : d;
  return __builtin_sqrtf(s > 0.0f ? s : 0.0f);
}

// Whether a kept w at delta(w, v) = dwv leaves v, at delta(u, v) = duv,
// selectable: RNG (Algorithm 5) duv < dwv; alpha-RNG duv < alpha^2 dwv;
// tau-MNG e(duv) < e(dwv) + 3 tau.  Each is non-decreasing in dwv, so a
// screen that brackets dwv in [lo, hi] decides the pair when the rule gives
// the same answer at both ends.
FGIM_DEV bool pair_keeps(const SelectArgs& a, float duv, float dwv) {
  if (a.rule == FGIM_SELECT_ALPHA) {
    const float lim = a.a2 * dwv;
    return duv < lim;
  }
  if (a.rule == FGIM_SELECT_TAU) {
    const float lim = euclid_of(dwv, a.metric) + a.t3;
    return euclid_of(duv, a.metric) < lim;
  }
  return duv < dwv;
}

template <int MMAX>
__global__ void __launch_bounds__(256) select_kernel(SelectArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  uint64_t* occl = reinterpret_cast<uint64_t*>(smem);       // k x 2 words
  uint32_t* vid = reinterpret_cast<uint32_t*>(occl + 2 * a.k);
  float* vd = reinterpret_cast<float*>(vid + a.k);
  uint32_t* tv = reinterpret_cast<uint32_t*>(vd + a.k);
  uint32_t* ctr = reinterpret_cast<uint32_t*>(smem + ((a.k * (16 + 12) + 15) / 16) * 16);  // 4 words
  float* rows = reinterpret_cast<float*>(ctr + 4);
  const uint32_t d = a.nc * 4 + 4;  // padded LDS row stride (spreads rows over banks)
  const int P = static_cast<int>(a.P), M = static_cast<int>(a.M);
  const int l = threadIdx.x % P;

  for (uint64_t u = blockIdx.x; u < a.N; u += gridDim.x) {
    if (threadIdx.x == 0) {
      ctr[0] = 0;
      ctr[1] = 0;
    }
    for (uint32_t t = threadIdx.x; t < a.k; t += 256) {
      const uint32_t v = a.ids[u * a.k + t];
      vid[t] = v;
      vd[t] = a.dist[u * a.k + t];
      tv[t] = v == kNone || !a.T ? 0u : a.T[v];
      occl[2 * t] = 0;
      occl[2 * t + 1] = 0;
      if (v != kNone) atomicMax(&ctr[1], t + 1);
    }
    __syncthreads();
    const uint32_t cnt = ctr[1];
    if (a.stage_rows) {
      for (uint32_t i = threadIdx.x; i < cnt * a.nc; i += 256) {
        const uint32_t e = i / a.nc, ch = i - e * a.nc;
        *reinterpret_cast<float4*>(rows + e * d + 4 * ch) =
            *reinterpret_cast<const float4*>(a.X + static_cast<uint64_t>(vid[e]) * a.ld + 4 * ch);
      }
      __syncthreads();
    }
    // occlusion tile: bit q of occl[p] set when delta(w_q, v_p) <= delta(u, v_p),
    // q < p; one P-lane group per row p (rows with T(v_p) = 1 are exempt).
    // Rows are dealt to groups statically and every loop that contains a
    // cross-lane shuffle is wave-uniform (inner trip count = the wave's
    // largest row, predicated per group).
    {
      const uint32_t G = 64 / P, g = (threadIdx.x % 64) / P, wave = threadIdx.x / 64;
      for (uint32_t base = wave * G; base < cnt; base += 4 * G) {
        const uint32_t pp = base + g;
        const bool act = pp < cnt && tv[pp] != 1u;
        const uint32_t qmax = min(base + G, cnt) - 1;  // largest row index of this wave's batch
        float4 x[MMAX];
        const float* xr = a.stage_rows ? (act ? rows + pp * d : rows)
                                       : a.X + (act ? static_cast<uint64_t>(vid[pp]) * a.ld : 0ull);
        load_row<MMAX>(x, xr, a.nc, P, M, l);
        const float dup = act ? vd[pp] : 0.0f;
        uint64_t m0 = 0, m1 = 0;
        for (uint32_t q = 0; q < qmax; ++q) {
          const bool valid = act && q < pp;
          const float* rw = a.stage_rows ? rows + q * d : a.X + static_cast<uint64_t>(vid[q]) * a.ld;
          const float dwv = pair_distance_x<MMAX>(x, rw, a.metric, a.nc, P, M, l, valid);
          if (valid && !pair_keeps(a, dup, dwv)) {
            if (q < 64) m0 |= 1ull << q;
            else m1 |= 1ull << (q - 64);
          }
        }
        if (act && l == 0) {
          occl[2 * pp] = m0;
          occl[2 * pp + 1] = m1;
        }
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      uint64_t kept0 = 0, kept1 = 0;
      uint32_t ns = 0;
      for (uint32_t p = 0; p < cnt && ns < a.R; ++p) {
        const bool keep = tv[p] == 1u || ((occl[2 * p] & kept0) == 0 && (occl[2 * p + 1] & kept1) == 0);
        if (keep) {
          if (p < 64) kept0 |= 1ull << p;
          else kept1 |= 1ull << (p - 64);
          a.sel_ids[u * a.R + ns] = vid[p];
          a.sel_dist[u * a.R + ns] = vd[p];
          ++ns;
        }
      }
      a.sel_n[u] = ns;
    }
    __syncthreads();
  }
}

constexpr uint32_t kSelMfmaMaxK = 64;
constexpr uint32_t kSelMfmaSlice = 256;  // dimensions staged in LDS at a time
constexpr int kSelTiles = 10;            // lower-triangle 16 x 16 tiles for 64 rows
constexpr size_t kSelMfmaHead = 64 * 8 * 2 + 64 * 4 * 2 + 68 * 4 + 64 * 4 * 3;

FGIM_DEV uint32_t select_bit64(uint64_t m, uint32_t r) {
  uint32_t pos = 0;
#pragma unroll
  for (uint32_t w = 32; w >= 1; w >>= 1) {
    const uint32_t c = static_cast<uint32_t>(__popcll(m & ((1ull << w) - 1ull)));
    if (r >= c) {
      r -= c;
      m >>= w;
      pos += w;
    }
  }
  return pos;
}

// Neighbour selection with the occlusion tile screened on MFMA, one
// wavefront per vertex (k <= 64 list entries).  The list's rows are staged
// in LDS as BF16, kSelMfmaSlice dimensions at a time, and the Gram tiles
// accumulate over the slices; every pair (w_q, v_p), q < p, gets
// the estimate of delta(w_q, v_p) and its bound (screen_estimate): the
// occlusion bit is set when the estimate plus the bound is below
// delta(u, v_p), left clear when the estimate minus the bound exceeds it,
// and otherwise decided by the canonical FP32 distance.  The bits are those
// of the plain computation.
constexpr uint32_t kSelStage = 2;  // row chunks a lane loads before staging them

template <int MMAX>
__global__ void __launch_bounds__(128) select_mfma_kernel(SelectArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int wave = threadIdx.x / 64;
  const int lane = lane_id();
  unsigned char* wbase = smem + static_cast<size_t>(wave) * a.wave_smem;
  uint64_t* occl = reinterpret_cast<uint64_t*>(wbase);   // bit q of row p: w_q occludes v_p
  uint64_t* unc = occl + 64;                             // bit q of row p: undecided by the screen
  uint32_t* vid = reinterpret_cast<uint32_t*>(unc + 64);
  uint32_t* tv = vid + 64;
  uint32_t* rowoff = tv + 64;                            // 65 prefix counts of undecided pairs
  float* vd = reinterpret_cast<float*>(rowoff + 68);
  float* nrm = vd + 64;
  float* qe = nrm + 64;
  uint16_t* rows = reinterpret_cast<uint16_t*>(qe + 64);  // BF16 rows, stride slice + 8
  const uint32_t slice = a.dpad < kSelMfmaSlice ? a.dpad : kSelMfmaSlice;
  const uint32_t srow = slice + 8;
  const uint32_t dim = a.nc * 4;
  const float gam = fp32_gamma(dim);
  const int P = static_cast<int>(a.P), M = static_cast<int>(a.M);
  const int l = lane % P, g = lane / P, G = 64 / P;

  for (uint64_t u = blockIdx.x * 2ull + wave; u < a.N; u += gridDim.x * 2ull) {
    const bool in = static_cast<uint32_t>(lane) < a.k;
    const uint32_t v = in ? a.ids[u * a.k + lane] : kNone;
    // the list's entries up to its first free slot
    const uint64_t invalid = ballot(v == kNone);
    const uint32_t cnt = invalid ? static_cast<uint32_t>(ffs64(invalid)) : 64u;
    const bool valid = static_cast<uint32_t>(lane) < cnt;
    vid[lane] = valid ? v : kNone;
    vd[lane] = valid ? a.dist[u * a.k + lane] : 0.0f;
    tv[lane] = valid && a.T ? a.T[v] : 0u;
    nrm[lane] = valid ? a.nrm2[v] : 0.0f;
    qe[lane] = valid ? sqrtf(a.qerr2[v]) * (1.0f + gam) * 1.0001f : 0.0f;
    occl[lane] = 0;
    unc[lane] = 0;
    wave_lds_sync();
    const uint32_t kpad = (cnt + 15) & ~15u;
    const uint32_t nt = kpad / 16;
    const uint32_t ntl = nt * (nt + 1) / 2;  // tiles (I, J), J <= I, in order t = I (I + 1) / 2 + J
    floatx4_t acc[kSelTiles];
#pragma unroll
    for (int t = 0; t < kSelTiles; ++t) acc[t] = floatx4_t{0.f, 0.f, 0.f, 0.f};
    for (uint32_t s0 = 0; s0 < a.dpad; s0 += slice) {
      const uint32_t sw = a.dpad - s0 < slice ? a.dpad - s0 : slice;  // multiple of 32
      const uint32_t per_row = sw / 8;
      const uint32_t total = kpad * per_row;
      // kSelStage chunks per lane are loaded before any is converted and
      // stored, so their memory latencies overlap
      for (uint32_t base = 0; base < total; base += 64 * kSelStage) {
        float4 f[kSelStage][2];
#pragma unroll
        for (uint32_t b = 0; b < kSelStage; ++b) {
          const uint32_t idx = base + b * 64 + lane;
          const uint32_t e = idx / per_row, t0 = s0 + 8 * (idx - e * per_row);
          f[b][0] = f[b][1] = make_float4(0.f, 0.f, 0.f, 0.f);
          if (idx < total && e < cnt && t0 < dim) {
            const float* xr = a.X + static_cast<uint64_t>(vid[e]) * a.ld + t0;
            f[b][0] = *reinterpret_cast<const float4*>(xr);
            if (t0 + 4 < dim) f[b][1] = *reinterpret_cast<const float4*>(xr + 4);
          }
        }
#pragma unroll
        for (uint32_t b = 0; b < kSelStage; ++b) {
          const uint32_t idx = base + b * 64 + lane;
          const uint32_t e = idx / per_row, c8 = 8 * (idx - e * per_row);
          const float4 f0 = f[b][0], f1 = f[b][1];
          shortx8_t v8;
          v8[0] = bf16_rne(f0.x); v8[1] = bf16_rne(f0.y); v8[2] = bf16_rne(f0.z); v8[3] = bf16_rne(f0.w);
          v8[4] = bf16_rne(f1.x); v8[5] = bf16_rne(f1.y); v8[6] = bf16_rne(f1.z); v8[7] = bf16_rne(f1.w);
          if (idx < total) *reinterpret_cast<shortx8_t*>(rows + e * srow + c8) = v8;
        }
      }
      wave_lds_sync();
      // D[i][j] = <row i, row j> over this slice, accumulated
#pragma unroll
      for (int t = 0; t < kSelTiles; ++t) {
        if (static_cast<uint32_t>(t) < ntl) {
          const uint32_t I = t >= 6 ? 3 : (t >= 3 ? 2 : (t >= 1 ? 1 : 0));
          const uint32_t J = static_cast<uint32_t>(t) - I * (I + 1) / 2;
          for (uint32_t kb = 0; kb < sw; kb += 32) {
            const shortx8_t ra = *reinterpret_cast<const shortx8_t*>(rows + (16 * I + lane % 16) * srow + kb + 8 * (lane / 16));
            const shortx8_t rb = *reinterpret_cast<const shortx8_t*>(rows + (16 * J + lane % 16) * srow + kb + 8 * (lane / 16));
            acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, ra),
                                                             __builtin_bit_cast(bf16x8_t, rb), acc[t], 0, 0, 0);
          }
        }
      }
      wave_lds_sync();
    }
#pragma unroll
    for (int t = 0; t < kSelTiles; ++t) {
      if (static_cast<uint32_t>(t) < ntl) {
        const uint32_t I = t >= 6 ? 3 : (t >= 3 ? 2 : (t >= 1 ? 1 : 0));
        const uint32_t J = static_cast<uint32_t>(t) - I * (I + 1) / 2;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const uint32_t i = 16 * I + 4 * (lane / 16) + r, j = 16 * J + lane % 16;
          if (i < cnt && j < i && tv[i] != 1u) {
            float dt, err;
            screen_estimate(acc[t][r], nrm[i], nrm[j], qe[i], qe[j], gam, a.metric, &dt, &err);
            const float dup = vd[i];
            // the exact delta(w_j, v_i) lies in [dt - err, dt + err]
            if (!pair_keeps(a, dup, dt + err)) atomicOr(reinterpret_cast<unsigned long long*>(&occl[i]), 1ull << j);
            else if (!pair_keeps(a, dup, dt - err)) atomicOr(reinterpret_cast<unsigned long long*>(&unc[i]), 1ull << j);
          }
        }
      }
    }
    wave_lds_sync();
    // exact re-scoring of the undecided pairs, enumerated flat over rows
    {
      const uint32_t c0 = static_cast<uint32_t>(lane) < cnt ? static_cast<uint32_t>(__popcll(unc[lane])) : 0u;
      uint32_t incl = c0;
#pragma unroll
      for (int st = 1; st < 64; st <<= 1) {
        const uint32_t o = static_cast<uint32_t>(__shfl_up(static_cast<int>(incl), st, 64));
        if (lane >= st) incl += o;
      }
      rowoff[lane + 1] = incl;
      if (lane == 0) rowoff[0] = 0;
    }
    wave_lds_sync();
    const uint32_t nu = rowoff[cnt];
    for (uint32_t b = 0; b < nu; b += static_cast<uint32_t>(G)) {
      const uint32_t idx = b + static_cast<uint32_t>(g);
      const bool act = idx < nu;
      uint32_t i = 0, j = 0;
      if (act) {
        uint32_t lo = 0, hi = cnt;  // the row holding idx: last row with rowoff <= idx
        while (hi - lo > 1) {
          const uint32_t mid = (lo + hi) / 2;
          if (rowoff[mid] <= idx) lo = mid;
          else hi = mid;
        }
        i = lo;
        j = select_bit64(unc[i], idx - rowoff[i]);
      }
      const float dd = pair_distance<MMAX>(a.X + static_cast<uint64_t>(vid[i]) * a.ld,
                                           a.X + static_cast<uint64_t>(vid[j]) * a.ld, a.metric, a.nc, P, M, l, act);
      if (act && l == 0 && !pair_keeps(a, vd[i], dd)) atomicOr(reinterpret_cast<unsigned long long*>(&occl[i]), 1ull << j);
    }
    wave_lds_sync();
    if (lane == 0) {
      uint64_t kept = 0;
      uint32_t ns = 0;
      for (uint32_t p = 0; p < cnt && ns < a.R; ++p) {
        if (tv[p] == 1u || (occl[p] & kept) == 0) {
          kept |= 1ull << p;
          a.sel_ids[u * a.R + ns] = vid[p];
          a.sel_dist[u * a.R + ns] = vd[p];
          ++ns;
        }
      }
      a.sel_n[u] = ns;
    }
    wave_lds_sync();
  }
}

__global__ void sel_count_kernel(const uint32_t* sel_ids, const uint32_t* sel_n, uint64_t N, uint32_t R, uint32_t* cnt) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < N * R;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    if (i % R < sel_n[i / R]) atomicAdd(&cnt[sel_ids[i]], 1u);
}

__global__ void sel_scatter_kernel(const uint32_t* sel_ids, const float* sel_dist, const uint32_t* sel_n, uint64_t N,
                                   uint32_t R, uint32_t* cur, uint64_t* rev) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < N * R;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    if (i % R >= sel_n[i / R]) continue;
    const uint32_t pos = atomicAdd(&cur[sel_ids[i]], 1u);
    rev[pos] = make_key(sel_dist[i], static_cast<uint32_t>(i / R));
  }
}

template <int NR>
__global__ void __launch_bounds__(256) fill_kernel(const uint32_t* sel_ids, const float* sel_dist, const uint32_t* sel_n,
                                                   const uint32_t* roff, const uint64_t* rev, uint64_t N, uint32_t R,
                                                   uint32_t* pg_ids, uint32_t* pg_deg) {
  const uint64_t nw = gridDim.x * 4ull;
  for (uint64_t u = blockIdx.x * 4ull + threadIdx.x / 64; u < N; u += nw) {
    Pool<NR> out;
    out.clear();
    const uint32_t ns = sel_n[u];
    for (uint32_t b = 0; b < ns; b += 64) {
      const uint32_t t = b + lane_id();
      const uint64_t ck = t < ns ? make_key(sel_dist[u * R + t], sel_ids[u * R + t]) : kSentinel;
      out.insert_batch(ck, R);
    }
    const uint32_t b0 = roff[u], b1 = roff[u + 1];
    for (uint32_t b = b0; b < b1; b += 64) {
      const uint64_t ck = b + lane_id() < b1 ? rev[b + lane_id()] : kSentinel;
      out.insert_batch(ck, R);
    }
    uint32_t deg = 0;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const uint32_t e = r * 64 + lane_id();
      deg += popc64(ballot(e < R && out.key[r] != kSentinel));
      if (e < R) pg_ids[u * R + e] = out.key[r] == kSentinel ? kNone : key_id(out.key[r]);
    }
    if (lane_id() == 0) pg_deg[u] = deg;
  }
}

// every id < N or FGIM_NONE, and FGIM_NONE only as padding after a list's
// entries (k ids per list)
__global__ void validate_lists_kernel(const uint32_t* ids, uint64_t nk, uint64_t N, uint32_t k, uint32_t* err) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < nk;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint32_t v = ids[i];
    if (v == kNone) continue;
    if (v >= N || (i % k != 0 && ids[i - 1] == kNone)) atomicOr(err, 1u);
  }
}

static uint32_t grid_n(uint64_t n, uint32_t per_block = 256) {
  const uint64_t b = (n + per_block - 1) / per_block;
  return static_cast<uint32_t>(std::min<uint64_t>(std::max<uint64_t>(b, 1), 65536));
}

static uint32_t pow2_ceil(uint32_t x) {
  uint32_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

// Neighbour selection (Algorithm 5's first step, or a swap-in rule) over
// `rows` lists of width k (ids index the n_x rows of X; T nullable: no
// indegree exemption), up to R per list, into sel_ids / sel_dist (rows x R)
// and sel_n.  nrm2 / qerr2 (the MFMA screen's row norms over all n_x rows)
// are computed into scratch when null and the screen runs.
fgim_status select_lists(const float* X, uint64_t n_x, uint64_t ld, uint32_t dim, int metric, uint64_t rows,
                         uint32_t k, uint32_t R, const uint32_t* ids, const float* dist, const uint32_t* T,
                         uint32_t rule, float param, uint32_t flags, const float* nrm2_in, const float* qerr2_in,
                         uint32_t* sel_ids, float* sel_dist, uint32_t* sel_n, Scratch& scr, hipStream_t s) {
  if (rows == 0) return FGIM_OK;
  const uint64_t N = rows;
  const uint32_t nc = dim / 4, Nch = pow2_ceil(nc);
  const uint32_t P = std::min<uint32_t>(64, std::max<uint32_t>(std::min<uint32_t>(4, Nch), Nch / 4));
  const uint32_t M = Nch / P;
  const size_t head = ((k * (16 + 12) + 15) / 16) * 16 + 16;
  const size_t rows_b = static_cast<size_t>(k) * (dim + 4) * 4;
  const bool stage = head + rows_b <= 96 * 1024;
  const size_t smem = head + (stage ? rows_b : 0);
  const float a2 = param * param;   // rounded once, as the rule states
  const float t3 = 3.0f * param;
  SelectArgs sa{X, ld, nc, metric, N, k, R, ids, dist, T, sel_ids, sel_dist, sel_n, P, M, stage,
                nullptr, nullptr, 0, 0, rule, a2, t3};
  const uint32_t grid = static_cast<uint32_t>(std::min<uint64_t>(N, static_cast<uint64_t>(device_cus()) * 8));
  const uint32_t dpad = (dim + 31) / 32 * 32;
  const bool use_mfma = k <= kSelMfmaMaxK && !(flags & FGIM_FLAG_NO_MFMA_SCREEN);
  if (use_mfma) {
    const float* nrm2 = nrm2_in;
    const float* qerr2 = qerr2_in;
    if (!nrm2 || !qerr2) {
      float *n2 = nullptr, *q2 = nullptr;
      FGIM_TRY(scr.get(&n2, n_x));
      FGIM_TRY(scr.get(&q2, n_x));
      HIP_TRY(launch_row_norms(X, n_x, dim, ld, n2, q2, s));
      nrm2 = n2;
      qerr2 = q2;
    }
    sa.nrm2 = nrm2;
    sa.qerr2 = qerr2;
    sa.dpad = dpad;
    const uint32_t kpad = (static_cast<uint32_t>(k) + 15) & ~15u;
    const uint32_t slice = std::min(dpad, kSelMfmaSlice);
    sa.wave_smem = static_cast<uint32_t>(kSelMfmaHead + static_cast<size_t>(kpad) * (slice + 8) * 2);
    const size_t msmem = 2 * static_cast<size_t>(sa.wave_smem);
    const uint32_t mgrid = static_cast<uint32_t>(std::min<uint64_t>((N + 1) / 2, static_cast<uint64_t>(device_cus()) * 16));
    auto kern = M <= 4 ? select_mfma_kernel<4> : select_mfma_kernel<16>;
    if (msmem > 64 * 1024)
      HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  static_cast<int>(msmem)));
    hipLaunchKernelGGL(kern, dim3(mgrid), dim3(128), msmem, s, sa);
  } else if (M <= 4) {
    if (smem > 64 * 1024)
      HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(select_kernel<4>), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  static_cast<int>(smem)));
    hipLaunchKernelGGL(select_kernel<4>, dim3(grid), dim3(256), smem, s, sa);
  } else {
    if (smem > 64 * 1024)
      HIP_TRY(hipFuncSetAttribute(reinterpret_cast<const void*>(select_kernel<16>), hipFuncAttributeMaxDynamicSharedMemorySize,
                                  static_cast<int>(smem)));
    hipLaunchKernelGGL(select_kernel<16>, dim3(grid), dim3(256), smem, s, sa);
  }
  HIP_TRY(hipGetLastError());
  return FGIM_OK;
}

// Stage 3.  Lists from a caller are checked first (ids in range, no entry
// after a free slot); the merge passes its own refined lists as trusted
// and skips the check and its host wait.
fgim_status prune_impl(const fgim_dataset* d, const fgim_params* p, const uint32_t* ids, const float* dist,
                       const uint32_t* T, uint32_t* pg_ids, uint32_t* pg_deg, hipStream_t s, bool trusted) {
  FGIM_TRY(check_dataset(d, false));
  if (!p) return fail(FGIM_ERR_INVALID_ARG, "params is NULL");
  if (!ids || !dist || !T || !pg_ids || !pg_deg) return fail(FGIM_ERR_INVALID_ARG, "NULL buffer");
  if (p->k == 0 || p->k > FGIM_MAX_K) return fail(FGIM_ERR_INVALID_ARG, "k = %u out of 1..%u", p->k, FGIM_MAX_K);
  if (p->R == 0 || p->R > FGIM_MAX_K) return fail(FGIM_ERR_INVALID_ARG, "R = %u out of 1..%u", p->R, FGIM_MAX_K);
  const uint64_t N = d->n_total, k = p->k, R = p->R;
  if (N * std::max(k, R) >= 0xFFFFFFFFull) return fail(FGIM_ERR_UNSUPPORTED, "N x max(k, R) exceeds 32-bit offsets");
  if (p->select_rule > FGIM_SELECT_TAU) return fail(FGIM_ERR_INVALID_ARG, "unknown select_rule %u", p->select_rule);
  if (p->select_rule != FGIM_SELECT_RNG && d->metric == FGIM_IP)
    return fail(FGIM_ERR_INVALID_ARG, "alpha-RNG and tau-MNG need a metric distance (L2 or cosine); "
                                      "transform inner-product data with fgim_mips_to_l2");
  if (p->select_rule == FGIM_SELECT_ALPHA && !(p->select_param >= 1.0f))
    return fail(FGIM_ERR_INVALID_ARG, "alpha = %g must be >= 1", static_cast<double>(p->select_param));
  if (p->select_rule == FGIM_SELECT_TAU && !(p->select_param >= 0.0f && p->select_param < 1e30f))
    return fail(FGIM_ERR_INVALID_ARG, "tau = %g must be finite and >= 0", static_cast<double>(p->select_param));
  Scratch scr(s);
  uint32_t *sel_ids = nullptr, *sel_n = nullptr, *cnt = nullptr, *off = nullptr, *cur = nullptr, *tmp = nullptr,
           *err = nullptr;
  float* sel_dist = nullptr;
  uint64_t* rev = nullptr;
  FGIM_TRY(scr.get(&sel_ids, N * R));
  FGIM_TRY(scr.get(&sel_dist, N * R));
  FGIM_TRY(scr.get(&sel_n, N));
  FGIM_TRY(scr.get(&cnt, N + 1));
  FGIM_TRY(scr.get(&off, N + 1));
  FGIM_TRY(scr.get(&cur, N + 1));
  FGIM_TRY(scr.get(&rev, N * R));
  FGIM_TRY(scr.get(&tmp, scan_tmp_words(N) + 16));
  FGIM_TRY(scr.get(&err, 4));
  if (!trusted) {
    HIP_TRY(fill_u32(err, 0u, 1, s));
    hipLaunchKernelGGL(validate_lists_kernel, dim3(grid_n(N * k)), dim3(256), 0, s, ids, N * k, N, p->k, err);
    uint32_t herr = 0;
    HIP_TRY(hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (herr) return fail(FGIM_ERR_GRAPH, "a k-NN list holds an id >= n_total or an entry after a free slot");
  }
  FGIM_TRY(select_lists(d->base, N, d->ld, d->dim, d->metric, N, p->k, p->R, ids, dist, T, p->select_rule,
                        p->select_param, p->flags, nullptr, nullptr, sel_ids, sel_dist, sel_n, scr, s));
  HIP_TRY(hipGetLastError());
  HIP_TRY(fill_u32(cnt, 0u, N, s));
  hipLaunchKernelGGL(sel_count_kernel, dim3(grid_n(N * R)), dim3(256), 0, s, sel_ids, sel_n, N, p->R, cnt);
  HIP_TRY(exclusive_scan(cnt, off, N, tmp, s));
  HIP_TRY(hipMemcpyAsync(cur, off, 4 * N, hipMemcpyDeviceToDevice, s));
  hipLaunchKernelGGL(sel_scatter_kernel, dim3(grid_n(N * R)), dim3(256), 0, s, sel_ids, sel_dist, sel_n, N, p->R, cur, rev);
  if (R <= 64)
    hipLaunchKernelGGL(fill_kernel<1>, dim3(grid_n(N, 4)), dim3(256), 0, s, sel_ids, sel_dist, sel_n, off, rev, N, p->R,
                       pg_ids, pg_deg);
  else
    hipLaunchKernelGGL(fill_kernel<2>, dim3(grid_n(N, 4)), dim3(256), 0, s, sel_ids, sel_dist, sel_n, off, rev, N, p->R,
                       pg_ids, pg_deg);
  HIP_TRY(hipGetLastError());
  return FGIM_OK;
}

// smallest retained global id in [lo, hi) (FGIM_NONE when none): atomicMin
__global__ void first_valid_kernel(const uint8_t* valid, uint64_t lo, uint64_t hi, uint32_t* out) {
  uint32_t best = kNone;
  for (uint64_t g = lo + blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; g < hi;
       g += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    if (valid[g] && static_cast<uint32_t>(g) < best) {
      best = static_cast<uint32_t>(g);
      break;
    }
  if (best != kNone) atomicMin(out, best);
}

// The merged graph's entry: the entry of the largest sub-index (lowest
// index on ties); with validity flags, the smallest retained id of that
// sub-index when its entry is dropped, passing over sub-indexes with no
// retained vertex.  `word` is a device word of scratch.
fgim_status merged_entry(const fgim_dataset* d, uint32_t* word, uint32_t* entry, hipStream_t s) {
  std::vector<uint32_t> order(d->h);
  for (uint32_t i = 0; i < d->h; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [d](uint32_t x, uint32_t y) { return d->subs[x].n > d->subs[y].n; });
  if (!d->valid) {
    *entry = static_cast<uint32_t>(d->subs[order[0]].row_offset + d->subs[order[0]].entry);
    return FGIM_OK;
  }
  for (uint32_t i : order) {
    const fgim_subindex& sb = d->subs[i];
    const uint64_t e = sb.row_offset + sb.entry;
    uint8_t ve = 0;
    HIP_TRY(hipMemcpyAsync(&ve, d->valid + e, 1, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (ve) {
      *entry = static_cast<uint32_t>(e);
      return FGIM_OK;
    }
    HIP_TRY(fill_u32(word, kNone, 1, s));
    const uint32_t blocks = static_cast<uint32_t>(std::min<uint64_t>((sb.n + 255) / 256, 4096));
    hipLaunchKernelGGL(first_valid_kernel, dim3(blocks), dim3(256), 0, s, d->valid, sb.row_offset,
                       sb.row_offset + sb.n, word);
    HIP_TRY(hipGetLastError());
    uint32_t hv = kNone;
    HIP_TRY(hipMemcpyAsync(&hv, word, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (hv != kNone) {
      *entry = hv;
      return FGIM_OK;
    }
  }
  *entry = kNone;
  return FGIM_OK;
}

fgim_status cross_query_impl(const fgim_dataset* d, const fgim_params* p, uint32_t* ids, float* dist,
                             fgim_stats* stats, hipStream_t s, uint32_t* L_used);
fgim_status refine_impl(const fgim_dataset* d, const fgim_params* p, uint32_t* ids, float* dist, uint32_t* T_out,
                        fgim_stats* stats, hipStream_t s, bool trusted);

}  // namespace fgim

using namespace fgim;

extern "C" {

fgim_status fgim_prune(const fgim_dataset* data, const fgim_params* params, const uint32_t* knn_ids,
                       const float* knn_dist, const uint32_t* indegree, uint32_t* pg_ids, uint32_t* pg_deg,
                       void* stream) {
  fail(FGIM_OK, "");
  return prune_impl(data, params, knn_ids, knn_dist, indegree, pg_ids, pg_deg, static_cast<hipStream_t>(stream), false);
}

fgim_status fgim_merge(const fgim_dataset* data, const fgim_params* params, uint32_t* pg_ids, uint32_t* pg_deg,
                       uint32_t* entry, fgim_stats* stats, void* stream) {
  fail(FGIM_OK, "");
  if (stats) memset(stats, 0, sizeof(*stats));
  hipStream_t s = static_cast<hipStream_t>(stream);
  FGIM_TRY(check_dataset(data, true));
  if (!params || !pg_ids || !pg_deg || !entry) return fail(FGIM_ERR_INVALID_ARG, "NULL argument");
  if (params->R == 0 || params->R > FGIM_MAX_K) return fail(FGIM_ERR_INVALID_ARG, "R = %u out of 1..%u", params->R, FGIM_MAX_K);
  const uint64_t N = data->n_total, k = params->k;
  Scratch scr(s);
  uint32_t *ids = nullptr, *T = nullptr;
  float* dist = nullptr;
  if (k == 0 || k > FGIM_MAX_K) return fail(FGIM_ERR_INVALID_ARG, "k = %u out of 1..%u", params->k, FGIM_MAX_K);
  uint32_t* word = nullptr;
  FGIM_TRY(scr.get(&ids, N * k));
  FGIM_TRY(scr.get(&dist, N * k));
  FGIM_TRY(scr.get(&T, N));
  FGIM_TRY(scr.get(&word, 1));
  hipEvent_t ev[4] = {};
  for (auto& e : ev) HIP_TRY(hipEventCreate(&e));
  HIP_TRY(hipEventRecord(ev[0], s));
  fgim_stats st1{}, st2{};
  FGIM_TRY(cross_query_impl(data, params, ids, dist, stats ? &st1 : nullptr, s, nullptr));
  HIP_TRY(hipEventRecord(ev[1], s));
  FGIM_TRY(refine_impl(data, params, ids, dist, T, stats ? &st2 : nullptr, s, true));
  HIP_TRY(hipEventRecord(ev[2], s));
  FGIM_TRY(prune_impl(data, params, ids, dist, T, pg_ids, pg_deg, s, true));
  HIP_TRY(hipEventRecord(ev[3], s));
  FGIM_TRY(merged_entry(data, word, entry, s));
  HIP_TRY(hipEventSynchronize(ev[3]));
  if (stats) {
    *stats = st1;
    for (int i = 0; i < 3; ++i) {
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, ev[i], ev[i + 1]));
      stats->ms_stage[i] = ms;
    }
    stats->proposals = st2.proposals;
    stats->repaired = st2.repaired;
    stats->rechecked = st2.rechecked;
    stats->repair_batches = st2.repair_batches;
    stats->repair_alone = st2.repair_alone;
    stats->refine_attempts = st2.refine_attempts;
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  return FGIM_OK;
}

}  // extern "C"
