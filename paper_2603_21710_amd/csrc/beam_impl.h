// Persistent wavefront-per-query beam search (Algorithm 1) and stage 1 of
// FGIM, PGs -> k-NNG (Section 4.1, Algorithm 2), for gfx950.
//
// One 64-lane wavefront owns one work item at a time and pops the next from
// a global queue.  Stage-1 item u: score u's local out-neighbours, run the
// beam search in every other sub-index, and fold everything into a running
// top-k; search item q: one beam search in one graph.
//
// The pool C (at most L <= 64*NR entries) lives in registers, sorted, one
// entry per lane per register, with an "expanded" bit.  The query row lives
// in registers too.  Each expansion reads one adjacency row (one id per
// lane, coalesced), filters ids through a per-wave visited cache in LDS,
// scores the new ids with P lanes per distance (coalesced float4 row
// gathers, canonical sum, xor-butterfly reduction) and inserts the keys that
// beat the current L-th entry.
//
// Visited cache.  The cache holds whole ids in two-choice slots and may
// forget ids (a new id overwrites an occupied slot when both of its slots
// are taken); it never reports an id that was not scored in this search.  Forgetting cannot change the result: a
// re-scored id is either still in the pool -- its key is identical, so the
// insertion sees a duplicate and drops it -- or it left the pool earlier,
// which means its key exceeded the L-th key at that time; the L-th key never
// increases, so the id is dropped again.  The pool evolves exactly as with
// an exact visited set, for any cache size.
#pragma once

#include "fgim_device.h"

namespace fgim {

struct SubDev {
  uint64_t off;
  const uint32_t* adj;
  uint32_t n;
  uint32_t stride;
  uint32_t entry;
  uint32_t pad_;
};

enum RowFmt : int { kF32 = 0, kBF16 = 1, kFP8 = 2 };

struct BeamArgs {
  const float* X;          // FP32 rows (query rows in stage 1, re-ranking)
  uint64_t ld;
  uint32_t nc;             // chunks of 4 coordinates (dim / 4)
  int metric;
  const uint16_t* xb;      // BF16 copy (dense, dim per row) or null
  const uint8_t* x8;       // FP8 copy or null
  const float* x8s;        // FP8 scales
  uint32_t dim;
  const SubDev* subs;
  uint32_t h;
  uint32_t L;
  uint32_t k;              // top-k of stage 1 / results kept by a search
  uint32_t rerank;         // entries per search re-scored in FP32 (low precision)
  uint64_t n_items;
  uint64_t item_stride;    // stage-1 item t is vertex t * item_stride (1: every vertex)
  int compact_out;         // 1: stage-1 item t writes output row t instead of row u
  uint32_t* out_ids;
  float* out_dist;
  uint32_t* counter;       // work-queue head, zero at launch
  const uint32_t* err;     // non-zero: a graph failed validation; do nothing
  unsigned long long* stats;  // ndc, expansions, searches (nullable)
  uint32_t vis_log2;       // visited-cache slots = 1 << vis_log2
  uint32_t P;              // lanes per distance
  uint32_t M;              // chunks per lane = padded chunk count / P
  int search_mode;         // 1: items are rows of Q searched in subs[0]
  const float* Q;
  uint64_t ldq;
  const uint8_t* valid;    // phi's validity flag per global id (null: all valid)
  const uint32_t* entries; // search items: per-query entry point (null: subs[0].entry)
};

struct WaveLds {
  uint32_t* vis;
  uint32_t* cand;   // 64 ids (rows relative to the graph offset)
  uint64_t* ckey;   // 64 keys
};

template <int NR>
struct Pool {
  uint64_t key[NR];
  uint32_t exp;     // bit r: entry r*64+lane is expanded

  FGIM_DEV void clear() {
#pragma unroll
    for (int r = 0; r < NR; ++r) key[r] = kSentinel;
    exp = 0;
  }

  // key of entry `cap-1`, the one a new key has to beat
  FGIM_DEV uint64_t theta(uint32_t cap) const {
    uint32_t e = cap - 1;
    uint64_t v = kSentinel;
#pragma unroll
    for (int r = 0; r < NR; ++r)
      if (static_cast<uint32_t>(r) == e / 64) v = readlane64(key[r], e % 64);
    return v;
  }

  // Insert uniform key c keeping the first `cap` entries; c is dropped when
  // it is already present (same id => same key) or does not make the cut.
  // The inserted entry's flag bit is `flag`.
  FGIM_DEV void insert(uint64_t c, uint32_t cap, uint32_t flag = 0) {
    int pos = 0;
    bool dup = false;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      pos += popc64(ballot(key[r] < c));
      dup |= ballot(key[r] == c) != 0;
    }
    if (dup || static_cast<uint32_t>(pos) >= cap) return;
    uint64_t carry = kSentinel;
    uint32_t carry_exp = 0;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      uint64_t last = readlane64(key[r], 63);
      uint32_t expr = (exp >> r) & 1u;
      uint32_t last_exp = readlane(expr, 63);
      uint64_t up = shift_up64(key[r], carry);
      uint32_t up_exp = shift_up32(expr, carry_exp);
      int e = r * 64 + lane_id();
      uint64_t nk = e < pos ? key[r] : (e == pos ? c : up);
      uint32_t ne = e < pos ? expr : (e == pos ? flag : up_exp);
      if (static_cast<uint32_t>(e) >= cap) {
        nk = kSentinel;
        ne = 0;
      }
      key[r] = nk;
      exp = (exp & ~(1u << r)) | (ne << r);
      carry = last;
      carry_exp = last_exp;
    }
  }

  // insert every lane's candidate key (kSentinel = none) that beats theta
  FGIM_DEV int insert_batch(uint64_t ck, uint32_t cap, uint32_t flag = 0) {
    int n = 0;
    uint64_t th = theta(cap);
    uint64_t mask = ballot(ck < th);
    while (mask) {
      int j = ffs64(mask);
      uint64_t c = readlane64(ck, j);
      insert(c, cap, flag);
      ++n;
      if (lane_id() == j) ck = kSentinel;
      th = theta(cap);
      mask = ballot(ck < th);
    }
    return n;
  }

  // position of the first unexpanded entry, or -1
  FGIM_DEV int first_unexpanded() const {
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      uint64_t m = ballot(key[r] != kSentinel && !((exp >> r) & 1u));
      if (m) return r * 64 + ffs64(m);
    }
    return -1;
  }

  FGIM_DEV uint64_t at(int pos) const {
    uint64_t v = kSentinel;
#pragma unroll
    for (int r = 0; r < NR; ++r)
      if (r == pos / 64) v = readlane64(key[r], pos % 64);
    return v;
  }

  FGIM_DEV void mark_expanded(int pos) {
    if (lane_id() == pos % 64) exp |= 1u << (pos / 64);
  }
};

// Score candidates cand[0..m) (row ids relative to `goff`) against the query
// held in q; key = (delta, key_off + id).  Group g of P lanes scores
// candidates g, g+G, ... (G = 64/P).  The rows of U consecutive group
// batches (at most UCAP) are loaded before any is reduced, so their memory
// latencies overlap.  All lanes must call this.
template <bool L2, int MMAX, int UCAP = 3, class Row>
FGIM_DEV void score_batch(const Row& rows, uint64_t goff, uint32_t key_off, const float4 (&q)[MMAX],
                          const BeamArgs& a, const WaveLds& lds, int m) {
  // group batches in flight: one for FP32 rows (95 VGPRs, 20 resident waves
  // per CU: 9 % faster than two batches at 16 waves on 8 uneven sub-indexes
  // of 2 M rows, d = 96, within 1.3 % elsewhere), else as many as about 32
  // registers of raw (BF16 / FP8) row data per lane hold, at most three for
  // BF16 (four take the kernel past 128 VGPRs, to 12 resident waves per CU,
  // and measured 12-25 % slower on d = 96, 128 and 768) and four for FP8
  // (122 VGPRs: 3.7 % faster at d = 768, level at d = 96 and 128; five
  // reach 130 VGPRs and are 20-28 % slower)
  constexpr int kRawRegs = static_cast<int>(sizeof(typename Row::Raw) / 4);
  constexpr int kRawCap = kRawRegs == 1 ? 4 : 3;
  constexpr int kLowP = 32 / (MMAX * kRawRegs) < kRawCap ? 32 / (MMAX * kRawRegs) : kRawCap;
  constexpr int U0 = MMAX > 4 ? 1 : (kRawRegs == 4 ? 1 : kLowP);
  constexpr int U = U0 < UCAP ? U0 : UCAP;
  const int P = static_cast<int>(a.P);
  const int M = static_cast<int>(a.M);
  const int G = 64 / P;
  const int g = lane_id() / P;
  const int l = lane_id() % P;
  for (int base = 0; base < m; base += G * U) {
    typename Row::Raw rv[U][MMAX];
    float sc[U];
    uint32_t rid[U];
    // batches past the last candidate are skipped (wave-uniform): an
    // expansion brings about as many new ids as a vertex has neighbours,
    // often fewer than G * U
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (base + u * G >= m) break;
      const int c = base + u * G + g;
      const bool act = c < m;
      rid[u] = lds.cand[act ? c : 0];
      sc[u] = act ? rows.scale(goff + rid[u]) : 1.0f;
#pragma unroll
      for (int mi = 0; mi < MMAX; ++mi) {
        const uint32_t ch = static_cast<uint32_t>(l + mi * P);
        rv[u][mi] = (mi < M && act && ch < a.nc) ? rows.raw(goff + rid[u], ch) : typename Row::Raw{};
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (base + u * G >= m) break;
      const int c = base + u * G + g;
      const bool act = c < m;
      float s[MMAX];
#pragma unroll
      for (int mi = 0; mi < MMAX; ++mi) {
        s[mi] = 0.0f;
        const uint32_t ch = static_cast<uint32_t>(l + mi * P);
        if (mi < M && act && ch < a.nc) s[mi] = chunk_sum<L2 ? kL2 : kIP>(q[mi], Row::decode(rv[u][mi], sc[u]));
      }
      const float d = finish_metric(reduce_chunk_sums<MMAX>(s, P, M), a.metric);
      if (act && l == 0) lds.ckey[c] = make_key(d, key_off + rid[u]);
    }
  }
}

// The visited cache holds whole ids in two-choice slots: an id is seen when
// either of its slots holds it, and a new id takes its first slot if free,
// else its second if free, else its first.  Two choices forget far fewer
// ids than one at the same size; a forgotten id is only scored again.
FGIM_DEV uint32_t vis_slot(uint32_t v, uint32_t log2) {
  return (v * 2654435761u) >> (32 - log2);
}

FGIM_DEV uint32_t vis_slot2(uint32_t v, uint32_t log2) {
  return ((v ^ 0x5bd1e995u) * 0x85ebca6bu) >> (32 - log2);
}

// Algorithm 1 from ep on the graph whose rows start at goff; leaves the
// final pool (keys with local ids) in `pool`.
template <bool L2, int MMAX, int NR, class Row>
FGIM_DEV void beam_search(Pool<NR>& pool, const Row& rows, uint64_t goff, const uint32_t* adj,
                          uint32_t stride, uint32_t ep, const float4 (&q)[MMAX], const BeamArgs& a,
                          const WaveLds& lds, unsigned long long& ndc, unsigned long long& nexp) {
  const uint32_t S = 1u << a.vis_log2;
  for (uint32_t i = lane_id(); i < S; i += 64) lds.vis[i] = kNone;
  if (lane_id() == 0) {
    lds.vis[vis_slot(ep, a.vis_log2)] = ep;
    lds.cand[0] = ep;
  }
  __syncthreads();
  score_batch<L2, MMAX, 1>(rows, goff, 0u, q, a, lds, 1);
  __syncthreads();
  pool.clear();
  {
    uint64_t k0 = lds.ckey[0];
    if (lane_id() == 0) pool.key[0] = k0;
  }
  ndc += 1;
  for (;;) {
    const int pos = pool.first_unexpanded();
    if (pos < 0) break;
    pool.mark_expanded(pos);
    nexp += 1;
    const uint32_t u = key_id(pool.at(pos));
    for (uint32_t t0 = 0; t0 < stride; t0 += 64) {
      const uint32_t t = t0 + lane_id();
      uint32_t v = t < stride ? adj[static_cast<uint64_t>(u) * stride + t] : kNone;
      const bool valid = v != kNone;
      const uint32_t s1 = valid ? vis_slot(v, a.vis_log2) : 0u;
      const uint32_t s2 = valid ? vis_slot2(v, a.vis_log2) : 0u;
      const uint32_t c1 = lds.vis[s1], c2 = lds.vis[s2];
      const bool seen = valid && (c1 == v || c2 == v);
      const bool isnew = valid && !seen;
      if (isnew) lds.vis[c1 != kNone && c2 == kNone ? s2 : s1] = v;
      const uint64_t nm = ballot(isnew);
      const int m = popc64(nm);
      if (m == 0) continue;
      if (isnew) lds.cand[mbcnt(nm)] = v;
      __syncthreads();
      // two raw batches, not three, beside a two-register pool: that keeps
      // the BF16 / FP8 instances at 124 VGPRs (16 resident waves per CU
      // instead of 12) and measured 18-19 % faster at L = 96 (d = 96, 128)
      score_batch<L2, MMAX, (NR >= 2 ? 2 : 4)>(rows, goff, 0u, q, a, lds, m);
      __syncthreads();
      ndc += static_cast<unsigned long long>(m);
      const uint64_t ck = lane_id() < m ? lds.ckey[lane_id()] : kSentinel;
      pool.insert_batch(ck, a.L);
      __syncthreads();
    }
  }
}

template <bool L2, int MMAX>
FGIM_DEV void load_query(float4 (&q)[MMAX], const float* row, const BeamArgs& a) {
  const int P = static_cast<int>(a.P);
  const int l = lane_id() % P;
#pragma unroll
  for (int mi = 0; mi < MMAX; ++mi) {
    const uint32_t ch = static_cast<uint32_t>(l + mi * P);
    if (mi < static_cast<int>(a.M) && ch < a.nc)
      q[mi] = *reinterpret_cast<const float4*>(row + 4ull * ch);
    else
      q[mi] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
}

constexpr uint32_t kItemsPerPop = 1;

template <bool L2, int FMT, int NR, int MMAX>
__global__ void __launch_bounds__(64) beam_kernel(BeamArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  WaveLds lds;
  lds.ckey = reinterpret_cast<uint64_t*>(smem);
  lds.cand = reinterpret_cast<uint32_t*>(smem + 64 * sizeof(uint64_t));
  lds.vis = lds.cand + 64;
  if (*a.err != 0u) return;

  RowF32 f32rows{a.X, a.ld};
  unsigned long long ndc = 0, nexp = 0, nsearch = 0;
  Pool<NR> pool;
  Pool<NR> topk;
  float4 q[MMAX];

  // items are popped kItemsPerPop at a time (more than one per pop measured
  // slower on 2 x 500k rows: the tail imbalance outweighs the atomics saved)
  uint32_t next = 0, left = 0;
  for (;;) {
    if (left == 0) {
      uint32_t b = 0;
      if (lane_id() == 0) b = atomicAdd(a.counter, kItemsPerPop);
      next = uniform(shfl_u(b, 0));
      left = kItemsPerPop;
    }
    const uint32_t item = next++;
    --left;
    if (item >= a.n_items) break;

    if (a.search_mode) {
      const SubDev g = a.subs[0];
      load_query<L2, MMAX>(q, a.Q + static_cast<uint64_t>(item) * a.ldq, a);
      const uint32_t ep = a.entries ? a.entries[item] : g.entry;
      if (FMT == kF32) {
        beam_search<L2, MMAX, NR>(pool, f32rows, g.off, g.adj, g.stride, ep, q, a, lds, ndc, nexp);
      } else if (FMT == kBF16) {
        RowBF16 rb{a.xb, a.dim};
        beam_search<L2, MMAX, NR>(pool, rb, g.off, g.adj, g.stride, ep, q, a, lds, ndc, nexp);
      } else {
        RowFP8 r8{a.x8, a.x8s, a.dim};
        beam_search<L2, MMAX, NR>(pool, r8, g.off, g.adj, g.stride, ep, q, a, lds, ndc, nexp);
      }
      nsearch += 1;
#pragma unroll
      for (int r = 0; r < NR; ++r) {
        const uint32_t e = r * 64 + lane_id();
        if (e < a.k) {
          const uint64_t kk = pool.key[r];
          a.out_ids[static_cast<uint64_t>(item) * a.k + e] = kk == kSentinel ? kNone : key_id(kk);
          a.out_dist[static_cast<uint64_t>(item) * a.k + e] = key_dist(kk);
        }
      }
      continue;
    }

    // ---- stage 1 item: global vertex u ----
    const uint64_t u = static_cast<uint64_t>(item) * a.item_stride;
    const uint64_t orow = a.compact_out ? item : u;
    if (a.valid && !a.valid[u]) {
      // phi drops u: no list, no searches
      for (uint32_t e = lane_id(); e < a.k; e += 64) {
        a.out_ids[orow * a.k + e] = kNone;
        a.out_dist[orow * a.k + e] = __builtin_inff();
      }
      continue;
    }
    uint32_t gi = 0;
    for (uint32_t i = 0; i < a.h; ++i)
      if (u >= a.subs[i].off) gi = i;
    const SubDev si = a.subs[gi];
    load_query<L2, MMAX>(q, a.X + u * a.ld, a);
    topk.clear();

    // local candidates C+(u): valid out-neighbours in G_i, scored on FP32 rows
    // (this and the re-ranking score one batch at a time: a second batch in
    // flight here took the BF16 / FP8 kernels past 128 VGPRs, to 12
    // resident waves per CU, 12 % slower on 2 x 500k rows, d = 768)
    const uint64_t lu = u - si.off;
    for (uint32_t t0 = 0; t0 < si.stride; t0 += 64) {
      const uint32_t t = t0 + lane_id();
      const uint32_t v = t < si.stride ? si.adj[lu * si.stride + t] : kNone;
      const bool valid = v != kNone && (!a.valid || a.valid[si.off + v]);
      const uint64_t nm = ballot(valid);
      const int m = popc64(nm);
      if (m == 0) continue;
      if (valid) lds.cand[mbcnt(nm)] = v;
      __syncthreads();
      score_batch<L2, MMAX, 1>(f32rows, si.off, static_cast<uint32_t>(si.off), q, a, lds, m);
      __syncthreads();
      const uint64_t ck = lane_id() < m ? lds.ckey[lane_id()] : kSentinel;
      topk.insert_batch(ck, a.k);
      __syncthreads();
    }

    // cross candidates C-(u): Algorithm 1 in every other G_j
    for (uint32_t j = 0; j < a.h; ++j) {
      if (j == gi) continue;
      const SubDev sj = a.subs[j];
      if (FMT == kF32) {
        beam_search<L2, MMAX, NR>(pool, f32rows, sj.off, sj.adj, sj.stride, sj.entry, q, a, lds, ndc, nexp);
      } else if (FMT == kBF16) {
        RowBF16 rb{a.xb, a.dim};
        beam_search<L2, MMAX, NR>(pool, rb, sj.off, sj.adj, sj.stride, sj.entry, q, a, lds, ndc, nexp);
      } else {
        RowFP8 r8{a.x8, a.x8s, a.dim};
        beam_search<L2, MMAX, NR>(pool, r8, sj.off, sj.adj, sj.stride, sj.entry, q, a, lds, ndc, nexp);
      }
      nsearch += 1;
      if (FMT == kF32) {
        // FP32 keys: fold the search's results as global ids -- its first
        // min(L, k) entries, or with validity flags every valid entry (the
        // running top-k keeps the best k either way)
        const uint32_t lim = a.valid ? a.L : a.k;
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const uint32_t e = r * 64 + lane_id();
          uint64_t ck = pool.key[r];
          if (e >= lim || ck == kSentinel || (a.valid && !a.valid[sj.off + key_id(ck)])) ck = kSentinel;
          else ck = (ck & 0xFFFFFFFF00000000ull) | static_cast<uint32_t>(sj.off + key_id(ck));
          topk.insert_batch(ck, a.k);
        }
      } else {
        // low-precision keys: re-score the first `rerank` (valid) entries on
        // FP32 rows
        uint32_t seen = 0;  // valid entries in the earlier registers
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const uint64_t pk = pool.key[r];
          const bool ok = pk != kSentinel && (!a.valid || a.valid[sj.off + key_id(pk)]);
          const uint64_t vm = ballot(ok);
          const bool take = ok && seen + static_cast<uint32_t>(mbcnt(vm)) < a.rerank;
          seen += static_cast<uint32_t>(popc64(vm));
          const uint64_t nm = ballot(take);
          const int m = popc64(nm);
          if (m == 0) continue;
          if (take) lds.cand[mbcnt(nm)] = key_id(pk);
          __syncthreads();
          score_batch<L2, MMAX, 1>(f32rows, sj.off, static_cast<uint32_t>(sj.off), q, a, lds, m);
          __syncthreads();
          const uint64_t ck = lane_id() < m ? lds.ckey[lane_id()] : kSentinel;
          topk.insert_batch(ck, a.k);
          __syncthreads();
        }
      }
    }

#pragma unroll
    for (int r = 0; r < NR; ++r) {
      const uint32_t e = r * 64 + lane_id();
      if (e < a.k) {
        const uint64_t kk = topk.key[r];
        a.out_ids[orow * a.k + e] = kk == kSentinel ? kNone : key_id(kk);
        a.out_dist[orow * a.k + e] = key_dist(kk);
      }
    }
  }

  if (a.stats && lane_id() == 0) {
    atomicAdd(&a.stats[0], ndc);
    atomicAdd(&a.stats[1], nexp);
    atomicAdd(&a.stats[2], nsearch);
  }
}

}  // namespace fgim
