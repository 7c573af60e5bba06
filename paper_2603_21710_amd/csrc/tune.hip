// Stage-1 tuner.
//
// The launch shape of the beam kernel (lanes per distance, resident waves per
// CU, visited-cache slots) changes no result bit, so it is chosen by timing
// trial launches on a strided sample of the vertices.  In the batched (h > 2)
// and low-precision forms the tuner may also lower the beam width L, never
// below the minimum-querying bound of Section 4.1.2 (enough cross candidates
// to fill k with the fewest local ones): it takes the smallest L whose k-NN
// lists on a sample keep at least 99 % of the ids found at the configured L.
//
// Decisions are kept in a text cache, one "key value" line each (a later line
// wins), at $FGIM_TUNE_CACHE (set but empty: memory only), else
// $XDG_CACHE_HOME/fgim/tune.txt, else $HOME/.cache/fgim/tune.txt.  An
// unreadable or unwritable cache only costs re-tuning.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <sys/stat.h>

#include <algorithm>
#include <chrono>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "fgim.h"
#include "fgim_internal.h"
#include "host_util.h"

namespace fgim {
namespace {

constexpr uint64_t kShapeSearches = 131072;    // searches per shape trial (h - 1 per vertex)
constexpr uint64_t kShapeMinVertices = 8192;   // ... from at least this many vertices
constexpr uint64_t kWidthSample = 16384;       // vertices per beam-width trial
constexpr double kWidthAgreement = 0.99;   // share of the configured-L ids kept

std::mutex g_mu;
std::map<std::string, std::string> g_cache;
std::string g_cache_file;
bool g_cache_read = false;

std::string cache_path() {
  if (const char* e = getenv("FGIM_TUNE_CACHE")) return e;
  const char* x = getenv("XDG_CACHE_HOME");
  if (x && *x) return std::string(x) + "/fgim/tune.txt";
  const char* h = getenv("HOME");
  if (h && *h) return std::string(h) + "/.cache/fgim/tune.txt";
  return std::string();
}

// (re)reads the cache file when the configured path changed
void sync_locked(const std::string& path) {
  if (g_cache_read && path == g_cache_file) return;
  g_cache.clear();
  g_cache_read = true;
  g_cache_file = path;
  if (path.empty()) return;
  FILE* f = fopen(path.c_str(), "r");
  if (!f) return;
  char line[1024];
  while (fgets(line, sizeof(line), f)) {
    line[strcspn(line, "\r\n")] = 0;
    char* sp = strchr(line, ' ');
    if (!sp || sp == line) continue;
    *sp = 0;
    g_cache[line] = sp + 1;
  }
  fclose(f);
}

bool cache_get(const std::string& key, std::string* val) {
  std::lock_guard<std::mutex> lock(g_mu);
  sync_locked(cache_path());
  auto it = g_cache.find(key);
  if (it == g_cache.end()) return false;
  *val = it->second;
  return true;
}

void cache_put(const std::string& key, const std::string& val) {
  std::lock_guard<std::mutex> lock(g_mu);
  const std::string path = cache_path();
  sync_locked(path);
  g_cache[key] = val;
  if (path.empty()) return;
  for (size_t i = 1; i < path.size(); ++i)
    if (path[i] == '/') (void)mkdir(path.substr(0, i).c_str(), 0755);
  FILE* f = fopen(path.c_str(), "a");
  if (!f) return;
  fprintf(f, "%s %s\n", key.c_str(), val.c_str());
  fclose(f);
}

std::string device_tag() {
  int dev = 0;
  hipDeviceProp_t pr;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&pr, dev) != hipSuccess) return "unknown";
  std::string arch(pr.gcnArchName);
  for (char& c : arch)
    if (c == ' ' || c == '/') c = '_';
  return arch + "/" + std::to_string(pr.multiProcessorCount);
}

// FNV-1a over the sub-index layout (sizes, strides, entries)
uint64_t layout_hash(const fgim_dataset* d) {
  uint64_t hsh = 1469598103934665603ull;
  auto mix = [&](uint64_t v) {
    for (int b = 0; b < 8; ++b) {
      hsh ^= (v >> (8 * b)) & 0xFF;
      hsh *= 1099511628211ull;
    }
  };
  for (uint32_t i = 0; i < d->h; ++i) {
    mix(d->subs[i].n);
    mix(d->subs[i].adj_stride);
    mix(d->subs[i].entry);
  }
  return hsh;
}

// vertices a shape trial searches from: about kShapeSearches searches
uint64_t shape_sample(const fgim_dataset* d) {
  const uint64_t per = d->h > 1 ? d->h - 1 : 1;
  return std::min<uint64_t>(d->n_total, std::max<uint64_t>(kShapeMinVertices, kShapeSearches / per));
}

uint32_t pow2_at_least(uint32_t x) {
  uint32_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

uint32_t log2_floor(uint64_t x) {
  uint32_t l = 0;
  while (x >> (l + 1)) ++l;
  return l;
}

struct Events {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  ~Events() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
};

// one launch over the sample that `a` describes
fgim_status trial(BeamArgs a, bool l2, int fmt, const BeamShape& sh, hipStream_t s, Events& ev, float* ms) {
  a.vis_log2 = sh.vis_log2;
  a.P = sh.P;
  a.M = sh.M;
  HIP_TRY(fill_u32(a.counter, 0u, 1, s));
  HIP_TRY(hipEventRecord(ev.e0, s));
  HIP_TRY(launch_beam(a, l2, fmt, sh, s));
  HIP_TRY(hipEventRecord(ev.e1, s));
  HIP_TRY(hipEventSynchronize(ev.e1));
  HIP_TRY(hipEventElapsedTime(ms, ev.e0, ev.e1));
  return FGIM_OK;
}

// share of the reference lists' ids that `got` also holds (rows of k ids)
double agreement(const std::vector<uint32_t>& ref, const std::vector<uint32_t>& got, uint32_t k) {
  uint64_t hit = 0, total = 0;
  std::vector<uint32_t> row(k);
  for (size_t r = 0; r * k < ref.size(); ++r) {
    std::copy(got.begin() + r * k, got.begin() + (r + 1) * k, row.begin());
    std::sort(row.begin(), row.end());
    for (uint32_t e = 0; e < k; ++e) {
      const uint32_t v = ref[r * k + e];
      if (v == FGIM_NONE) continue;
      ++total;
      hit += std::binary_search(row.begin(), row.end(), v) ? 1 : 0;
    }
  }
  return total ? static_cast<double>(hit) / static_cast<double>(total) : 1.0;
}

// smallest L in [lo, p->L] whose sampled lists keep kWidthAgreement of the
// configured-L ids (binary search; the configured L always qualifies)
fgim_status tune_width(BeamArgs a, const fgim_dataset* d, const fgim_params* p, int fmt, bool l2, uint32_t lo,
                       uint32_t* L, bool* ran, hipStream_t s, Events& ev) {
  char key[512];
  snprintf(key, sizeof(key), "width/%s/n%llu/h%u/d%u/m%d/f%d/k%u/L%u/rr%u/g%016llx", device_tag().c_str(),
           (unsigned long long)d->n_total, d->h, d->dim, (int)d->metric, fmt, p->k, p->L, p->rerank,
           (unsigned long long)layout_hash(d));
  std::string v;
  unsigned got = 0;
  if (cache_get(key, &v) && sscanf(v.c_str(), "%u", &got) == 1 && got >= lo && got <= p->L) {
    *L = got;
    return FGIM_OK;
  }
  *ran = true;
  const uint64_t S = std::min<uint64_t>(d->n_total, kWidthSample);
  a.n_items = S;
  a.item_stride = d->n_total / S;
  std::vector<uint32_t> ref(S * p->k), cur(S * p->k);
  auto run = [&](uint32_t Lc, std::vector<uint32_t>* out) -> fgim_status {
    BeamShape sh;
    FGIM_TRY(beam_shape(d->dim, Lc, p->k, p, &sh));
    a.L = Lc;
    FGIM_TRY(rerank_for(p, Lc, &a.rerank));
    float ms = 0.f;
    FGIM_TRY(trial(a, l2, fmt, sh, s, ev, &ms));
    HIP_TRY(hipMemcpyAsync(out->data(), a.out_ids, out->size() * 4, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return FGIM_OK;
  };
  FGIM_TRY(run(p->L, &ref));
  uint32_t lo_b = lo, hi_b = p->L;
  while (lo_b < hi_b) {
    const uint32_t mid = lo_b + (hi_b - lo_b) / 2;
    FGIM_TRY(run(mid, &cur));
    if (agreement(ref, cur, p->k) >= kWidthAgreement) hi_b = mid;
    else lo_b = mid + 1;
  }
  *L = hi_b;
  cache_put(key, std::to_string(hi_b));
  return FGIM_OK;
}

// fastest launch shape for width L among the fields p leaves at 0
fgim_status tune_shape(BeamArgs a, const fgim_dataset* d, const fgim_params* p, int fmt, bool l2, uint32_t L,
                       BeamShape* out, bool* ran, hipStream_t s, Events& ev) {
  char key[512];
  snprintf(key, sizeof(key), "shape/%s/d%u/f%d/l2%d/h%u/n%u/L%u/k%u/rr%u/P%u/w%u/v%u", device_tag().c_str(), d->dim,
           fmt, l2 ? 1 : 0, d->h, log2_floor(d->n_total), L, p->k, p->rerank, p->lanes_per_dist, p->waves_per_cu,
           p->visited_slots);
  std::string v;
  unsigned cP = 0, cw = 0, cv = 0;
  if (cache_get(key, &v) && sscanf(v.c_str(), "%u %u %u", &cP, &cw, &cv) == 3) {
    fgim_params q = *p;
    q.lanes_per_dist = cP;
    q.waves_per_cu = cw;
    q.visited_slots = cv;
    if (beam_shape(d->dim, L, p->k, &q, out) == FGIM_OK) return FGIM_OK;
  }
  *ran = true;
  const uint64_t S = shape_sample(d);
  a.n_items = S;
  a.item_stride = d->n_total / S;
  a.L = L;
  FGIM_TRY(rerank_for(p, L, &a.rerank));

  const uint32_t N = pow2_at_least(d->dim / 4);
  std::vector<uint32_t> Ps, Ws, Vs;
  if (p->lanes_per_dist) Ps.push_back(p->lanes_per_dist);
  else
    for (uint32_t P = 1; P <= 64; P <<= 1)
      if (P <= N && N / P <= 16 && P * 8 >= N) Ps.push_back(P);
  // 24 waves per CU never differed from 32 by more than noise, and 512 slots
  // never won: they are left out of the grid
  if (p->waves_per_cu) Ws.push_back(p->waves_per_cu);
  else Ws = {16, 32};
  if (p->visited_slots) Vs.push_back(p->visited_slots);
  else Vs = {1024, 2048, 4096};

  struct Cand {
    float ms;
    uint32_t P, w, v;
  };
  std::vector<Cand> cands;
  for (uint32_t P : Ps)
    for (uint32_t w : Ws)
      for (uint32_t vs : Vs) {
        fgim_params q = *p;
        q.lanes_per_dist = P;
        q.waves_per_cu = w;
        q.visited_slots = vs;
        BeamShape sh;
        if (beam_shape(d->dim, L, p->k, &q, &sh) != FGIM_OK) continue;
        float ms = 0.f;
        FGIM_TRY(trial(a, l2, fmt, sh, s, ev, &ms));
        cands.push_back(Cand{ms, P, w, vs});
      }
  if (cands.empty()) return fail(FGIM_ERR_INVALID_ARG, "no valid beam launch shape for dim %u", d->dim);
  // the first launch of each instance pays its load: re-time the leaders
  std::sort(cands.begin(), cands.end(), [](const Cand& x, const Cand& y) { return x.ms < y.ms; });
  const size_t top = std::min<size_t>(cands.size(), 4);
  for (size_t i = 0; i < top; ++i) {
    fgim_params q = *p;
    q.lanes_per_dist = cands[i].P;
    q.waves_per_cu = cands[i].w;
    q.visited_slots = cands[i].v;
    BeamShape sh;
    FGIM_TRY(beam_shape(d->dim, L, p->k, &q, &sh));
    for (int rep = 0; rep < 2; ++rep) {
      float ms = 0.f;
      FGIM_TRY(trial(a, l2, fmt, sh, s, ev, &ms));
      cands[i].ms = rep == 0 ? ms : std::min(cands[i].ms, ms);
    }
  }
  std::sort(cands.begin(), cands.begin() + top, [](const Cand& x, const Cand& y) { return x.ms < y.ms; });
  fgim_params q = *p;
  q.lanes_per_dist = cands[0].P;
  q.waves_per_cu = cands[0].w;
  q.visited_slots = cands[0].v;
  FGIM_TRY(beam_shape(d->dim, L, p->k, &q, out));
  char val[64];
  snprintf(val, sizeof(val), "%u %u %u", cands[0].P, cands[0].w, cands[0].v);
  cache_put(key, val);
  return FGIM_OK;
}

}  // namespace

fgim_status tune_stage1(const BeamArgs& a0, const fgim_dataset* d, const fgim_params* p, int fmt, bool l2,
                        uint32_t lo, uint32_t* L, BeamShape* shape, double* ms_tune, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  bool ran = false;
  Events ev;
  HIP_TRY(hipEventCreate(&ev.e0));
  HIP_TRY(hipEventCreate(&ev.e1));
  Scratch scr(s);
  const uint64_t S = std::max(shape_sample(d), std::min<uint64_t>(d->n_total, kWidthSample));
  BeamArgs a = a0;
  FGIM_TRY(scr.get(&a.out_ids, S * p->k));
  FGIM_TRY(scr.get(&a.out_dist, S * p->k));
  a.compact_out = 1;
  a.stats = nullptr;

  uint32_t width = p->L;
  if ((p->precision != FGIM_FP32 || d->h > 2) && lo < p->L)
    FGIM_TRY(tune_width(a, d, p, fmt, l2, lo, &width, &ran, s, ev));
  FGIM_TRY(tune_shape(a, d, p, fmt, l2, width, shape, &ran, s, ev));
  HIP_TRY(fill_u32(a0.counter, 0u, 1, s));
  *L = width;
  *ms_tune = ran ? std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() : 0.0;
  return FGIM_OK;
}

}  // namespace fgim
