// HNSW-adaptive merging (Section 4.3.3): the upper layers of an HNSW index
// rebuilt over the merged base graph, and the search over the hierarchy.
//
// The paper re-inserts every vertex of level >= 1 into the upper layers by
// HNSW's own incremental procedure.  The layers hold N/M, N/M^2, ...
// vertices, so here each layer is built in one batch from exact candidates:
//   members  V_l = {v : level[v] >= l} in ascending id (mask, scan, scatter)
//   cand     the ef nearest other members of every member, exact
//            (layer_knn_kernel: one wavefront per member, canonical FP32
//            distances, running top-ef)
//   sel      HNSW's neighbour heuristic (the RNG rule, no indegree
//            exemption) up to M, by the stage-3 selection kernels
//   uni      sel plus the reverse of every selection, first 2M by (delta, id)
//            (bidirectional edges; union_kernel)
//   adj      the heuristic again over uni, up to M (the pruning HNSW applies
//            to neighbours that gained an edge)
// The search descends greedily from the top entry through the layers
// (descent_kernel) and runs Algorithm 1 on the base graph from the vertex it
// reaches (the beam kernel with per-query entry points).
#include "fgim_internal.h"
#include "graph_util.h"
#include "host_util.h"

namespace fgim {

__global__ void level_mask_kernel(const uint8_t* level, uint64_t n, uint32_t l, uint32_t max_level,
                                  uint32_t* mask, uint32_t* err) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    const uint32_t lv = level[i];
    mask[i] = lv >= l ? 1u : 0u;
    if (lv > max_level) atomicOr(err, 1u);
  }
}

// members in ascending id, and the row of every member in the layer
__global__ void level_compact_kernel(const uint32_t* mask, const uint32_t* pos, uint64_t n, uint32_t* ids) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    if (mask[i]) ids[pos[i]] = static_cast<uint32_t>(i);
}

struct LayerArgs {
  BeamArgs b;              // rows (X, ld, nc, metric), P, M of the scorer
  const uint32_t* ids;     // members, ascending
  uint64_t n;              // member count
  uint32_t ef;
  uint32_t* cand_ids;      // n x ef
  float* cand_dist;
  uint32_t* counter;       // work-queue head, zero at launch
};

// Exact ef nearest other members of every member, one wavefront per member
// (popped from a queue): the member rows are scored against the member's
// row 64 at a time and folded into a running top-ef.
template <bool L2, int NR, int MMAX>
__global__ void __launch_bounds__(64) layer_knn_kernel(LayerArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  WaveLds lds;
  lds.ckey = reinterpret_cast<uint64_t*>(smem);
  lds.cand = reinterpret_cast<uint32_t*>(smem + 64 * sizeof(uint64_t));
  lds.vis = nullptr;
  RowF32 rows{a.b.X, a.b.ld};
  Pool<NR> top;
  float4 q[MMAX];
  for (;;) {
    uint32_t it = 0;
    if (lane_id() == 0) it = atomicAdd(a.counter, 1u);
    const uint64_t item = uniform(shfl_u(it, 0));
    if (item >= a.n) break;
    const uint32_t u = a.ids[item];
    load_query<L2, MMAX>(q, a.b.X + static_cast<uint64_t>(u) * a.b.ld, a.b);
    top.clear();
    for (uint64_t c0 = 0; c0 < a.n; c0 += 64) {
      const int m = static_cast<int>(a.n - c0 < 64 ? a.n - c0 : 64);
      if (lane_id() < m) lds.cand[lane_id()] = a.ids[c0 + lane_id()];
      __syncthreads();
      score_batch<L2, MMAX>(rows, 0, 0u, q, a.b, lds, m);
      __syncthreads();
      uint64_t ck = lane_id() < m ? lds.ckey[lane_id()] : kSentinel;
      if (ck != kSentinel && key_id(ck) == u) ck = kSentinel;
      top.insert_batch(ck, a.ef);
      __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const uint32_t e = r * 64 + lane_id();
      if (e < a.ef) {
        const uint64_t kk = top.key[r];
        a.cand_ids[item * a.ef + e] = kk == kSentinel ? kNone : key_id(kk);
        a.cand_dist[item * a.ef + e] = key_dist(kk);
      }
    }
  }
}

// reverse of every selection: the selecting member's global id, under the
// row of the selected one
__global__ void rev_count_kernel(const uint32_t* sel_ids, const uint32_t* sel_n, uint64_t n, uint32_t M,
                                 const uint32_t* pos, uint32_t* cnt) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n * M;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    if (i % M < sel_n[i / M]) atomicAdd(&cnt[pos[sel_ids[i]]], 1u);
}

__global__ void rev_fill_kernel(const uint32_t* sel_ids, const float* sel_dist, const uint32_t* sel_n, uint64_t n,
                                uint32_t M, const uint32_t* pos, const uint32_t* ids, uint32_t* cur, uint64_t* rev) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n * M;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
    if (i % M >= sel_n[i / M]) continue;
    const uint32_t at = atomicAdd(&cur[pos[sel_ids[i]]], 1u);
    rev[at] = make_key(sel_dist[i], ids[i / M]);
  }
}

// first 2M of sel(u) and its reverse edges, by (delta, id), one wavefront
// per member
template <int NR>
__global__ void __launch_bounds__(256) union_kernel(const uint32_t* sel_ids, const float* sel_dist,
                                                    const uint32_t* sel_n, const uint32_t* roff, const uint64_t* rev,
                                                    uint64_t n, uint32_t M, uint32_t* uni_ids, float* uni_dist) {
  const uint32_t W = 2 * M;
  for (uint64_t a = blockIdx.x * 4ull + threadIdx.x / 64; a < n; a += gridDim.x * 4ull) {
    Pool<NR> out;
    out.clear();
    const uint32_t ns = sel_n[a];
    {
      const uint64_t ck = static_cast<uint32_t>(lane_id()) < ns
                              ? make_key(sel_dist[a * M + lane_id()], sel_ids[a * M + lane_id()])
                              : kSentinel;
      out.insert_batch(ck, W);
    }
    const uint32_t b0 = roff[a], b1 = roff[a + 1];
    for (uint32_t b = b0; b < b1; b += 64) {
      const uint64_t ck = b + lane_id() < b1 ? rev[b + lane_id()] : kSentinel;
      out.insert_batch(ck, W);
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const uint32_t e = r * 64 + lane_id();
      if (e < W) {
        uni_ids[a * W + e] = out.key[r] == kSentinel ? kNone : key_id(out.key[r]);
        uni_dist[a * W + e] = key_dist(out.key[r]);
      }
    }
  }
}

struct DescentArgs {
  BeamArgs b;                // rows, P, M of the scorer; b.Q / b.ldq: queries
  uint64_t nq;
  const uint32_t* layer_ids;  // concatenated layers 1..max_level
  const uint32_t* layer_adj;  // M per member
  const uint64_t* start;      // first row of each layer (index l, device)
  const uint64_t* count;      // members of each layer (index l, device)
  uint32_t max_level, M, top;
  uint32_t* entries;          // out: per query, the vertex the descent reaches
  uint32_t* counter;
};

FGIM_DEV uint64_t uniform64(uint64_t v) {
  return (static_cast<uint64_t>(uniform(static_cast<uint32_t>(v >> 32))) << 32) | uniform(static_cast<uint32_t>(v));
}

// Greedy descent, one wavefront per query: in each layer from the highest,
// move to the closest neighbour (by (delta, id)) while it beats the current
// vertex.  The result is stored by every lane (one address, one value): a
// lane-0 branch at the end of the loop body was merged by the compiler with
// the lane-0 branch of the next queue pop, which split the loop in two, so
// that lanes 1..63 re-entered the item broadcast without lane 0 and spun on
// a stale item for ever.  The values that decide branches and loop exits are
// made wave-uniform for the same reason.
template <bool L2, int MMAX>
__global__ void __launch_bounds__(64) descent_kernel(DescentArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  WaveLds lds;
  lds.ckey = reinterpret_cast<uint64_t*>(smem);
  lds.cand = reinterpret_cast<uint32_t*>(smem + 64 * sizeof(uint64_t));
  lds.vis = nullptr;
  RowF32 rows{a.b.X, a.b.ld};
  float4 q[MMAX];
  for (;;) {
    uint32_t it = 0;
    if (lane_id() == 0) it = atomicAdd(a.counter, 1u);
    const uint64_t item = uniform(shfl_u(it, 0));
    if (item >= a.nq) break;
    load_query<L2, MMAX>(q, a.b.Q + item * a.b.ldq, a.b);
    if (lane_id() == 0) lds.cand[0] = a.top;
    __syncthreads();
    score_batch<L2, MMAX, 1>(rows, 0, 0u, q, a.b, lds, 1);
    __syncthreads();
    uint64_t best = uniform64(lds.ckey[0]);
    __syncthreads();
    for (uint32_t l = a.max_level; l >= 1; --l) {
      const uint64_t n = uniform64(a.count[l]);
      const uint64_t first = uniform64(a.start[l]);
      const uint32_t* ids = a.layer_ids + first;
      for (uint32_t step = 0; step < 0x7FFFFFFFu && n > 0; ++step) {
        // row of the current vertex: binary search of the ascending members
        const uint32_t cur = key_id(best);
        uint64_t lo = 0, hi = n;
        while (lo < hi) {
          const uint64_t mid = (lo + hi) / 2;
          if (uniform(ids[mid]) < cur) lo = mid + 1;
          else hi = mid;
        }
        if (lo >= n) break;
        if (uniform(ids[lo]) != cur) break;
        const uint32_t* row = a.layer_adj + (first + lo) * a.M;
        const uint32_t v = static_cast<uint32_t>(lane_id()) < a.M ? row[lane_id()] : kNone;
        const uint64_t nm = ballot(v != kNone);
        const int m = popc64(nm);
        if (m == 0) break;
        if (v != kNone) lds.cand[mbcnt(nm)] = v;
        __syncthreads();
        score_batch<L2, MMAX, 1>(rows, 0, 0u, q, a.b, lds, m);
        __syncthreads();
        const uint64_t ck = lane_id() < m ? lds.ckey[lane_id()] : kSentinel;
        __syncthreads();
        uint64_t nb = best;
        uint64_t mask = ballot(ck < nb);
        while (mask) {
          nb = uniform64(readlane64(ck, ffs64(mask)));
          mask = ballot(ck < nb);
        }
        if (nb == best) break;
        best = nb;
      }
    }
    a.entries[item] = key_id(best);
  }
}

static uint32_t grid_of(uint64_t n, uint32_t per = 256) {
  return static_cast<uint32_t>(std::min<uint64_t>(std::max<uint64_t>((n + per - 1) / per, 1), 65536));
}

// the scorer's launch shape for rows of `dim` (lanes per distance, chunks
// per lane): the beam kernel's default
static fgim_status scorer(uint32_t dim, BeamShape* sh) { return beam_shape(dim, 64, 1, nullptr, sh); }

template <bool L2>
static hipError_t launch_knn(const LayerArgs& a, const BeamShape& sh, uint32_t nr, hipStream_t s) {
  const dim3 grid(device_cus() * 16);
  const size_t smem = 64 * 8 + 64 * 4;
  if (sh.mmax == 2) {
    if (nr == 1) hipLaunchKernelGGL((layer_knn_kernel<L2, 1, 2>), grid, dim3(64), smem, s, a);
    else hipLaunchKernelGGL((layer_knn_kernel<L2, 2, 2>), grid, dim3(64), smem, s, a);
  } else if (sh.mmax == 4) {
    if (nr == 1) hipLaunchKernelGGL((layer_knn_kernel<L2, 1, 4>), grid, dim3(64), smem, s, a);
    else hipLaunchKernelGGL((layer_knn_kernel<L2, 2, 4>), grid, dim3(64), smem, s, a);
  } else {
    if (nr == 1) hipLaunchKernelGGL((layer_knn_kernel<L2, 1, 16>), grid, dim3(64), smem, s, a);
    else hipLaunchKernelGGL((layer_knn_kernel<L2, 2, 16>), grid, dim3(64), smem, s, a);
  }
  return hipGetLastError();
}

template <bool L2>
static hipError_t launch_descent(const DescentArgs& a, const BeamShape& sh, hipStream_t s) {
  const dim3 grid(device_cus() * 16);
  const size_t smem = 64 * 8 + 64 * 4;
  if (sh.mmax == 2) hipLaunchKernelGGL((descent_kernel<L2, 2>), grid, dim3(64), smem, s, a);
  else if (sh.mmax == 4) hipLaunchKernelGGL((descent_kernel<L2, 4>), grid, dim3(64), smem, s, a);
  else hipLaunchKernelGGL((descent_kernel<L2, 16>), grid, dim3(64), smem, s, a);
  return hipGetLastError();
}

fgim_status check_rows(const float* base, uint64_t n, uint32_t dim, uint64_t ld);
hipError_t validate_graph(const uint32_t* adj, uint32_t n, uint32_t stride, uint32_t* err, hipStream_t s,
                          uint32_t* min_deg, double* edges, double weight);

// every id below n or FGIM_NONE (sets *err otherwise)
__global__ void ids_in_range_kernel(const uint32_t* ids, uint64_t count, uint64_t n, uint32_t* err) {
  for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < count;
       i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
    if (ids[i] != kNone && ids[i] >= n) atomicOr(err, 1u);
}

}  // namespace fgim

using namespace fgim;

extern "C" fgim_status fgim_hnsw_layers(const float* base, uint64_t n, uint32_t dim, uint64_t ld, fgim_metric metric,
                                        const uint8_t* levels, uint32_t max_level, uint32_t M, uint32_t ef,
                                        const uint64_t* layer_count, uint32_t* layer_ids, uint32_t* layer_adj,
                                        uint32_t* top, void* stream) {
  clear_error();
  hipStream_t s = static_cast<hipStream_t>(stream);
  FGIM_TRY(check_rows(base, n, dim, ld));
  if (metric != FGIM_L2 && metric != FGIM_IP && metric != FGIM_COSINE) return fail(FGIM_ERR_INVALID_ARG, "unknown metric");
  if (!levels || !layer_count || !top || (max_level && (!layer_ids || !layer_adj)))
    return fail(FGIM_ERR_INVALID_ARG, "NULL argument");
  if (max_level > 64) return fail(FGIM_ERR_INVALID_ARG, "max_level %u > 64", max_level);
  if (M == 0 || M > 64) return fail(FGIM_ERR_INVALID_ARG, "M = %u out of 1..64", M);
  if (ef < M || ef > 128) return fail(FGIM_ERR_INVALID_ARG, "ef = %u must be in M..128", ef);
  uint64_t rows = 0;
  for (uint32_t l = 0; l < max_level; ++l) {
    if (l && layer_count[l] > layer_count[l - 1])
      return fail(FGIM_ERR_INVALID_ARG, "layer %u holds more vertices than layer %u", l + 1, l);
    rows += layer_count[l];
  }
  if (layer_count[0] > n) return fail(FGIM_ERR_INVALID_ARG, "layer 1 holds more vertices than the base");
  BeamShape sh;
  FGIM_TRY(scorer(dim, &sh));
  *top = FGIM_NONE;
  if (max_level == 0) return FGIM_OK;

  Scratch scr(s);
  const uint64_t n1 = layer_count[0];
  uint32_t *mask = nullptr, *pos = nullptr, *tmp = nullptr, *hdr = nullptr, *cid = nullptr, *sel_ids = nullptr,
           *sel_n = nullptr, *cnt = nullptr, *roff = nullptr, *cur = nullptr, *uid = nullptr, *sel2_n = nullptr;
  float *cdd = nullptr, *sel_dist = nullptr, *udd = nullptr, *sel2_dist = nullptr, *nrm2 = nullptr, *qerr2 = nullptr;
  uint64_t* rev = nullptr;
  FGIM_TRY(scr.get(&mask, n + 1));
  FGIM_TRY(scr.get(&pos, n + 1));
  FGIM_TRY(scr.get(&tmp, scan_tmp_words(n + 1) + 16));
  FGIM_TRY(scr.get(&hdr, 8));
  FGIM_TRY(scr.get(&cid, n1 * ef));
  FGIM_TRY(scr.get(&cdd, n1 * ef));
  FGIM_TRY(scr.get(&sel_ids, n1 * M));
  FGIM_TRY(scr.get(&sel_dist, n1 * M));
  FGIM_TRY(scr.get(&sel_n, n1));
  FGIM_TRY(scr.get(&cnt, n1 + 1));
  FGIM_TRY(scr.get(&roff, n1 + 1));
  FGIM_TRY(scr.get(&cur, n1 + 1));
  FGIM_TRY(scr.get(&rev, n1 * M));
  FGIM_TRY(scr.get(&uid, n1 * 2 * M));
  FGIM_TRY(scr.get(&udd, n1 * 2 * M));
  FGIM_TRY(scr.get(&sel2_dist, n1 * M));
  FGIM_TRY(scr.get(&sel2_n, n1));
  FGIM_TRY(scr.get(&nrm2, n));
  FGIM_TRY(scr.get(&qerr2, n));
  HIP_TRY(launch_row_norms(base, n, dim, ld, nrm2, qerr2, s));
  HIP_TRY(fill_u32(layer_adj, kNone, rows * M, s));
  const bool l2 = metric == FGIM_L2;
  uint64_t off = 0;
  for (uint32_t l = 1; l <= max_level; ++l) {
    const uint64_t nl = layer_count[l - 1];
    HIP_TRY(fill_u32(hdr, 0u, 8, s));
    hipLaunchKernelGGL(level_mask_kernel, dim3(grid_of(n)), dim3(256), 0, s, levels, n, l, max_level, mask, hdr + 1);
    HIP_TRY(exclusive_scan(mask, pos, n, tmp, s));
    uint32_t hv[2] = {0, 0};
    HIP_TRY(hipMemcpyAsync(&hv[0], pos + n, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(&hv[1], hdr + 1, 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (hv[1]) return fail(FGIM_ERR_INVALID_ARG, "a level exceeds max_level = %u", max_level);
    if (hv[0] != nl)
      return fail(FGIM_ERR_INVALID_ARG, "layer %u: %u vertices have level >= %u, layer_count says %llu", l, hv[0], l,
                  static_cast<unsigned long long>(nl));
    if (nl == 0) continue;
    uint32_t* ids = layer_ids + off;
    hipLaunchKernelGGL(level_compact_kernel, dim3(grid_of(n)), dim3(256), 0, s, mask, pos, n, ids);
    // exact candidates
    LayerArgs la{};
    la.b.X = base;
    la.b.ld = ld;
    la.b.nc = dim / 4;
    la.b.metric = metric;
    la.b.P = sh.P;
    la.b.M = sh.M;
    la.ids = ids;
    la.n = nl;
    la.ef = ef;
    la.cand_ids = cid;
    la.cand_dist = cdd;
    la.counter = hdr;
    HIP_TRY(l2 ? launch_knn<true>(la, sh, ef > 64 ? 2 : 1, s) : launch_knn<false>(la, sh, ef > 64 ? 2 : 1, s));
    // heuristic, bidirectional union, heuristic again
    FGIM_TRY(select_lists(base, n, ld, dim, metric, nl, ef, M, cid, cdd, nullptr, FGIM_SELECT_RNG, 0.0f, 0, nrm2,
                          qerr2, sel_ids, sel_dist, sel_n, scr, s));
    HIP_TRY(fill_u32(cnt, 0u, nl, s));
    hipLaunchKernelGGL(rev_count_kernel, dim3(grid_of(nl * M)), dim3(256), 0, s, sel_ids, sel_n, nl, M, pos, cnt);
    HIP_TRY(exclusive_scan(cnt, roff, nl, tmp, s));
    HIP_TRY(hipMemcpyAsync(cur, roff, 4 * nl, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(rev_fill_kernel, dim3(grid_of(nl * M)), dim3(256), 0, s, sel_ids, sel_dist, sel_n, nl, M, pos,
                       ids, cur, rev);
    if (2 * M <= 64)
      hipLaunchKernelGGL(union_kernel<1>, dim3(grid_of(nl, 4)), dim3(256), 0, s, sel_ids, sel_dist, sel_n, roff, rev,
                         nl, M, uid, udd);
    else
      hipLaunchKernelGGL(union_kernel<2>, dim3(grid_of(nl, 4)), dim3(256), 0, s, sel_ids, sel_dist, sel_n, roff, rev,
                         nl, M, uid, udd);
    HIP_TRY(hipGetLastError());
    FGIM_TRY(select_lists(base, n, ld, dim, metric, nl, 2 * M, M, uid, udd, nullptr, FGIM_SELECT_RNG, 0.0f, 0, nrm2,
                          qerr2, layer_adj + off * M, sel2_dist, sel2_n, scr, s));
    HIP_TRY(hipMemcpyAsync(top, ids, 4, hipMemcpyDeviceToHost, s));
    off += nl;
  }
  HIP_TRY(hipStreamSynchronize(s));
  return FGIM_OK;
}

extern "C" fgim_status fgim_search_layers(const float* base, uint64_t n, uint32_t dim, uint64_t ld, fgim_metric metric,
                                          const uint32_t* base_adj, uint32_t stride, const uint32_t* layer_ids,
                                          const uint32_t* layer_adj, const uint64_t* layer_count, uint32_t max_level,
                                          uint32_t M, uint32_t top, const float* queries, uint64_t nq, uint64_t ldq,
                                          uint32_t L, uint32_t topk, uint32_t* out_ids, float* out_dist, void* stream) {
  clear_error();
  hipStream_t s = static_cast<hipStream_t>(stream);
  FGIM_TRY(check_rows(base, n, dim, ld));
  if (metric != FGIM_L2 && metric != FGIM_IP && metric != FGIM_COSINE) return fail(FGIM_ERR_INVALID_ARG, "unknown metric");
  if (!base_adj || stride == 0 || stride > FGIM_MAX_STRIDE) return fail(FGIM_ERR_INVALID_ARG, "bad base graph");
  if (max_level > 64 || (max_level && (!layer_ids || !layer_adj || !layer_count)) || M == 0 || M > 64)
    return fail(FGIM_ERR_INVALID_ARG, "bad layers");
  if (top >= n) return fail(FGIM_ERR_INVALID_ARG, "top %u >= n", top);
  if (nq == 0) return FGIM_OK;
  if (!queries || ldq < dim || ldq % 4 || reinterpret_cast<uintptr_t>(queries) % 16 || nq >= 0xFFF00000ull)
    return fail(FGIM_ERR_INVALID_ARG, "bad query matrix");
  if (L == 0 || L > FGIM_MAX_L || topk == 0 || topk > L || !out_ids || !out_dist)
    return fail(FGIM_ERR_INVALID_ARG, "need 1 <= topk <= L <= %u and outputs", FGIM_MAX_L);
  BeamShape sh;
  FGIM_TRY(beam_shape(dim, L, topk, nullptr, &sh));
  Scratch scr(s);
  uint32_t *hdr = nullptr, *entries = nullptr;
  uint64_t* meta = nullptr;
  SubDev* sub = nullptr;
  FGIM_TRY(scr.get(&hdr, 8));
  FGIM_TRY(scr.get(&entries, nq));
  FGIM_TRY(scr.get(&meta, 2 * 66));
  FGIM_TRY(scr.get(&sub, 1));
  uint64_t hm[2 * 66] = {0};
  uint64_t acc = 0;
  for (uint32_t l = 1; l <= max_level; ++l) {
    hm[l] = acc;                // start
    hm[66 + l] = layer_count[l - 1];
    acc += layer_count[l - 1];
  }
  HIP_TRY(hipMemcpyAsync(meta, hm, sizeof(hm), hipMemcpyHostToDevice, s));
  HIP_TRY(fill_u32(hdr, 0u, 8, s));
  // malformed inputs are rejected before any of their ids is followed
  HIP_TRY(validate_graph(base_adj, static_cast<uint32_t>(n), stride, hdr + 3, s, nullptr, nullptr, 1.0));
  if (acc) {
    hipLaunchKernelGGL(ids_in_range_kernel, dim3(grid_of(acc)), dim3(256), 0, s, layer_ids, acc, n, hdr + 3);
    hipLaunchKernelGGL(ids_in_range_kernel, dim3(grid_of(acc * M)), dim3(256), 0, s, layer_adj, acc * M, n, hdr + 3);
  }
  uint32_t herr = 0;
  HIP_TRY(hipMemcpyAsync(&herr, hdr + 3, 4, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (herr) return fail(FGIM_ERR_GRAPH, "a base or layer adjacency id is out of range, a self-loop or a duplicate");
  DescentArgs da{};
  da.b.X = base;
  da.b.ld = ld;
  da.b.nc = dim / 4;
  da.b.metric = metric;
  da.b.P = sh.P;
  da.b.M = sh.M;
  da.b.Q = queries;
  da.b.ldq = ldq;
  da.nq = nq;
  da.layer_ids = layer_ids;
  da.layer_adj = layer_adj;
  da.start = meta;
  da.count = meta + 66;
  da.max_level = max_level;
  da.M = M;
  da.top = top;
  da.entries = entries;
  da.counter = hdr;
  HIP_TRY(metric == FGIM_L2 ? launch_descent<true>(da, sh, s) : launch_descent<false>(da, sh, s));
  SubDev hs{0, base_adj, static_cast<uint32_t>(n), stride, top, 0};
  HIP_TRY(hipMemcpyAsync(sub, &hs, sizeof(hs), hipMemcpyHostToDevice, s));
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
  a.counter = hdr + 2;
  a.err = hdr + 3;
  a.vis_log2 = sh.vis_log2;
  a.P = sh.P;
  a.M = sh.M;
  a.search_mode = 1;
  a.Q = queries;
  a.ldq = ldq;
  a.entries = entries;
  HIP_TRY(launch_beam(a, metric == FGIM_L2, kF32, sh, s));
  HIP_TRY(hipStreamSynchronize(s));
  return FGIM_OK;
}
