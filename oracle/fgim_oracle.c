/*
 * FGIM merge oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow CPU implementation of the three stages of FGIM (Wu et al.,
 * "FGIM: a Fast Graph-based Indexes Merging Framework for Approximate
 * Nearest Neighbor Search", PACMMOD 2026), written from the paper to check
 * the GPU library against.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load it; the library never does.  It
 * shares no code with the GPU path.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared -pthread (no -ffast-math),
 * so that every float operation below is the IEEE operation written.
 *
 * Conventions (readings of places where the paper is silent):
 *  - delta is squared L2, -<a,b> (inner product) or 1-<a,b> (cosine on
 *    unit vectors), summed in FP32 in the canonical order of
 *    oracle_distance; -0 is canonicalised to +0.
 *  - Every sort, top-k, "closest" and "farthest" uses the total order
 *    (delta ascending, global id ascending).
 *  - Ids are uint32; 0xFFFFFFFF pads short lists, with distance +inf.
 *
 * Parallel loops split independent units (queries, nodes) over pthreads;
 * the thread count never changes a bit of any result.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_NONE 0xFFFFFFFFu
#define ORC_L2 0
#define ORC_IP 1
#define ORC_COS 2

#define FLAG_NEW 1u
#define FLAG_REPLACED 2u
/* A list entry (t -> v) recorded, at t's Visit while it was new, as a new
 * reverse link of v, and not yet consumed by a Visit of v (Section 4.2.1:
 * Visit records reverse links; the target's Visit moves them into Cn). */
#define FLAG_RNEW 4u
#define ENT_SNAPSHOT 0x100u   /* apply: the entry comes from the list itself */

/* neighbour-selection rules of stage 3 (Section 4.3.1) */
#define ORC_SEL_RNG 0     /* Algorithm 5: delta(u,v) < delta(w,v) */
#define ORC_SEL_ALPHA 1   /* alpha-RNG (Vamana's robust prune) */
#define ORC_SEL_TAU 2     /* tau-MNG (tau-monotonic graph) */

typedef struct {
    uint64_t off;          /* global id of local vertex 0 (phi_i offset) */
    uint32_t n;            /* |V_i| */
    uint32_t stride;       /* row stride of adj (R_in) */
    const uint32_t* adj;   /* n x stride local ids, ORC_NONE padded */
    uint32_t entry;        /* local id of ep_i */
} oracle_sub;

typedef struct {
    float d;
    uint32_t id;
    uint32_t flag;
} ent_t;

/* ------------------------------------------------------------------ */
/* Distance (delta, Section 2.1) in the canonical FP32 order.          */
/* ------------------------------------------------------------------ */

/*
 * The dimensions are cut into chunks of 4 consecutive coordinates.  Each
 * chunk is summed left to right with fused multiply-adds starting from +0;
 * the chunk count is padded with zero chunks to a power of two N, and the
 * chunk sums are combined by the stride tree
 *     for (st = N/2; st >= 1; st /= 2)  s[c] = s[c] + s[c + st],  c < st.
 * The final sum r becomes r (L2), -r (inner product) or 1 - r (cosine),
 * and +0.0f is added to turn -0 into +0.
 */
float oracle_distance(const float* a, const float* b, uint32_t dim, int metric)
{
    uint32_t nc = (dim + 3u) / 4u;
    uint32_t N = 1;
    while (N < nc) N <<= 1;
    float s[1024];
    for (uint32_t c = 0; c < N; ++c) {
        float acc = 0.0f;
        if (c < nc) {
            uint32_t t0 = 4u * c, t1 = t0 + 4u < dim ? t0 + 4u : dim;
            for (uint32_t t = t0; t < t1; ++t) {
                if (metric == ORC_L2) {
                    float e = a[t] - b[t];
                    acc = fmaf(e, e, acc);
                } else {
                    acc = fmaf(a[t], b[t], acc);
                }
            }
        }
        s[c] = acc;
    }
    for (uint32_t st = N / 2; st >= 1; st /= 2)
        for (uint32_t c = 0; c < st; ++c) s[c] = s[c] + s[c + st];
    float r = s[0], out;
    if (metric == ORC_L2) out = r;
    else if (metric == ORC_IP) out = -r;
    else out = 1.0f - r;
    return out + 0.0f;
}

static int ent_less(const ent_t* x, const ent_t* y)
{
    return x->d < y->d || (x->d == y->d && x->id < y->id);
}

static int ent_cmp(const void* pa, const void* pb)
{
    const ent_t* x = (const ent_t*)pa;
    const ent_t* y = (const ent_t*)pb;
    if (ent_less(x, y)) return -1;
    if (ent_less(y, x)) return 1;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Parallel-for over [0, n) with pthreads.                              */
/* ------------------------------------------------------------------ */
typedef void (*range_fn)(void* ctx, uint64_t begin, uint64_t end, int tid);

typedef struct {
    range_fn fn;
    void* ctx;
    uint64_t n;
    int nth;
    int tid;
} par_arg;

static void* par_body(void* p)
{
    par_arg* a = (par_arg*)p;
    uint64_t per = (a->n + (uint64_t)a->nth - 1) / (uint64_t)a->nth;
    uint64_t b = per * (uint64_t)a->tid, e = b + per;
    if (e > a->n) e = a->n;
    if (b < e) a->fn(a->ctx, b, e, a->tid);
    return NULL;
}

static void parallel_for(uint64_t n, int threads, range_fn fn, void* ctx)
{
    if (threads < 1) threads = 1;
    if ((uint64_t)threads > n) threads = n ? (int)n : 1;
    pthread_t th[256];
    par_arg args[256];
    if (threads > 256) threads = 256;
    for (int t = 0; t < threads; ++t) {
        args[t] = (par_arg){fn, ctx, n, threads, t};
        if (t) pthread_create(&th[t], NULL, par_body, &args[t]);
    }
    par_body(&args[0]);
    for (int t = 1; t < threads; ++t) pthread_join(th[t], NULL);
}

/* ------------------------------------------------------------------ */
/* Algorithm 1, KNNSearch(q, G, L, L, ep).                              */
/* ------------------------------------------------------------------ */

typedef struct {
    ent_t* pool;        /* capacity L + stride */
    uint8_t* visited;   /* n bytes, all zero between searches */
    uint32_t* touched;  /* ids whose visited byte is set */
} search_ws;

/*
 * Best-first beam search.  The pool C holds at most L entries sorted by
 * (delta, id), each flagged expanded or not.  Each step expands the first
 * unexpanded entry, inserts every out-neighbour whose distance has not been
 * computed yet, re-sorts and keeps the first L.  The search ends when every
 * pool entry is expanded.  "Visited" marks a vertex when its distance is
 * computed (at insertion), so no vertex enters C twice and no distance is
 * computed twice.  Returns the pool size; ndc / nexp count distance
 * computations and expansions.
 */
static uint32_t knn_search(const float* q, const float* Xj, uint64_t ld,
                           uint32_t dim, int metric, const uint32_t* adj,
                           uint32_t stride, uint32_t ep, uint32_t L,
                           search_ws* ws, uint64_t* ndc, uint64_t* nexp)
{
    ent_t* C = ws->pool;
    uint32_t cnt = 0, ntouch = 0;
    ws->visited[ep] = 1;
    ws->touched[ntouch++] = ep;
    C[cnt++] = (ent_t){oracle_distance(q, Xj + (uint64_t)ep * ld, dim, metric), ep, 0};
    *ndc += 1;
    for (;;) {
        uint32_t i = 0;
        while (i < cnt && C[i].flag) ++i;
        if (i == cnt) break;
        C[i].flag = 1;
        *nexp += 1;
        uint32_t u = C[i].id;
        for (uint32_t t = 0; t < stride; ++t) {
            uint32_t v = adj[(uint64_t)u * stride + t];
            if (v == ORC_NONE || ws->visited[v]) continue;
            ws->visited[v] = 1;
            ws->touched[ntouch++] = v;
            C[cnt++] = (ent_t){oracle_distance(q, Xj + (uint64_t)v * ld, dim, metric), v, 0};
            *ndc += 1;
        }
        qsort(C, cnt, sizeof(ent_t), ent_cmp);
        if (cnt > L) cnt = L;
    }
    for (uint32_t t = 0; t < ntouch; ++t) ws->visited[ws->touched[t]] = 0;
    return cnt;
}

static int ws_alloc(search_ws* ws, uint32_t L, uint32_t stride, uint32_t n)
{
    ws->pool = (ent_t*)malloc(sizeof(ent_t) * ((size_t)L + stride + 1));
    ws->visited = (uint8_t*)calloc(n ? n : 1, 1);
    ws->touched = (uint32_t*)malloc(sizeof(uint32_t) * ((size_t)n + 1));
    return ws->pool && ws->visited && ws->touched;
}

static void ws_free(search_ws* ws)
{
    free(ws->pool);
    free(ws->visited);
    free(ws->touched);
}

static int check_graph(const uint32_t* adj, uint32_t n, uint32_t stride, uint32_t ep)
{
    if (ep >= n) return 0;
    for (uint64_t i = 0; i < (uint64_t)n * stride; ++i)
        if (adj[i] != ORC_NONE && adj[i] >= n) return 0;
    return 1;
}

/* Single search, for tests of Algorithm 1 on its own.  Returns -1 on a
 * malformed graph, else the number of results written. */
int oracle_knn_search(const float* q, const float* Xj, uint64_t ld, uint32_t dim,
                      int metric, const uint32_t* adj, uint32_t n, uint32_t stride,
                      uint32_t ep, uint32_t L, uint32_t* out_ids, float* out_dist,
                      uint64_t* ndc, uint64_t* nexp)
{
    if (!check_graph(adj, n, stride, ep) || L == 0) return -1;
    search_ws ws;
    if (!ws_alloc(&ws, L, stride, n)) { ws_free(&ws); return -1; }
    uint64_t a = 0, b = 0;
    uint32_t cnt = knn_search(q, Xj, ld, dim, metric, adj, stride, ep, L, &ws, &a, &b);
    for (uint32_t i = 0; i < cnt; ++i) {
        out_ids[i] = ws.pool[i].id;
        out_dist[i] = ws.pool[i].d;
    }
    if (ndc) *ndc = a;
    if (nexp) *nexp = b;
    ws_free(&ws);
    return (int)cnt;
}

/* ------------------------------------------------------------------ */
/* Stage 1: PGs -> k-NNG (Algorithm 2) with cross-querying.             */
/* ------------------------------------------------------------------ */

static uint32_t sub_of(const oracle_sub* subs, uint32_t h, uint64_t gid)
{
    for (uint32_t i = 0; i < h; ++i)
        if (gid >= subs[i].off && gid < subs[i].off + subs[i].n) return i;
    return h;
}

typedef struct {
    const float* X;       /* FP32 base rows */
    const float* Xs;      /* rows the beam search scores (X, or a dequantised copy) */
    uint64_t ld;
    uint32_t dim;
    int metric;
    const oracle_sub* subs;
    uint32_t h;
    uint32_t k, L, rerank;
    const uint64_t* nodes;
    uint32_t* out_ids;
    float* out_dist;
    uint64_t* ndc_t;      /* per thread */
    uint64_t* exp_t;
    int* err_t;
    const uint8_t* valid; /* phi's validity flag per global id (NULL: all valid) */
} cq_ctx;

/*
 * For vertex u of G_i: the local candidates C+ are u's out-neighbours in
 * G_i; every other G_j (ascending j) is searched from its entry point with
 * pool L; the union is sorted, mapped to global ids by phi_j(v) = off_j + v
 * and cut to k.  When the beam scores rows of a low-precision copy (Xs !=
 * X), each search's first `rerank` results are re-scored on the FP32 rows
 * before they enter the union.
 *
 * phi's validity (Section 4.1.3): phi maps only retained vertices.  An
 * invalid u gets an empty list; an invalid vertex is never a candidate (not
 * in C+, not among a search's results), but the searches still route
 * through it, since it is part of G_j's structure.  A search's results are
 * the valid entries of its final pool, in pool order; with a low-precision
 * copy the first `rerank` of them are re-scored.
 */
static void cq_range(void* p, uint64_t b, uint64_t e, int tid)
{
    cq_ctx* c = (cq_ctx*)p;
    uint32_t maxn = 0, maxs = 0;
    for (uint32_t i = 0; i < c->h; ++i) {
        if (c->subs[i].n > maxn) maxn = c->subs[i].n;
        if (c->subs[i].stride > maxs) maxs = c->subs[i].stride;
    }
    search_ws ws;
    size_t ucap = (size_t)maxs + (size_t)c->h * c->L + 1;
    ent_t* U = (ent_t*)malloc(sizeof(ent_t) * ucap);
    if (!ws_alloc(&ws, c->L, maxs, maxn) || !U) {
        c->err_t[tid] = 1;
        ws_free(&ws);
        free(U);
        return;
    }
    for (uint64_t idx = b; idx < e; ++idx) {
        uint64_t u = c->nodes ? c->nodes[idx] : idx;
        uint32_t gi = sub_of(c->subs, c->h, u);
        if (gi >= c->h) { c->err_t[tid] = 1; continue; }
        if (c->valid && !c->valid[u]) {
            for (uint32_t t = 0; t < c->k; ++t) {
                c->out_ids[idx * c->k + t] = ORC_NONE;
                c->out_dist[idx * c->k + t] = INFINITY;
            }
            continue;
        }
        const oracle_sub* si = &c->subs[gi];
        const float* xu = c->X + u * c->ld;
        uint64_t lu = u - si->off;
        size_t nu = 0;
        for (uint32_t t = 0; t < si->stride; ++t) {
            uint32_t v = si->adj[lu * si->stride + t];
            if (v == ORC_NONE) continue;
            uint64_t gv = si->off + v;
            if (c->valid && !c->valid[gv]) continue;
            U[nu++] = (ent_t){oracle_distance(xu, c->X + gv * c->ld, c->dim, c->metric),
                              (uint32_t)gv, FLAG_NEW};
        }
        for (uint32_t j = 0; j < c->h; ++j) {
            if (j == gi) continue;
            const oracle_sub* sj = &c->subs[j];
            const float* Xj = c->Xs + sj->off * c->ld;
            uint32_t cnt = knn_search(xu, Xj, c->ld, c->dim, c->metric, sj->adj,
                                      sj->stride, sj->entry, c->L, &ws,
                                      &c->ndc_t[tid], &c->exp_t[tid]);
            uint32_t take = cnt, taken = 0;
            if (c->Xs != c->X && c->rerank < take) take = c->rerank;
            for (uint32_t t = 0; t < cnt && taken < take; ++t) {
                uint64_t gv = sj->off + ws.pool[t].id;
                if (c->valid && !c->valid[gv]) continue;
                float dv = ws.pool[t].d;
                if (c->Xs != c->X)
                    dv = oracle_distance(xu, c->X + gv * c->ld, c->dim, c->metric);
                U[nu++] = (ent_t){dv, (uint32_t)gv, FLAG_NEW};
                ++taken;
            }
        }
        qsort(U, nu, sizeof(ent_t), ent_cmp);
        for (uint32_t t = 0; t < c->k; ++t) {
            c->out_ids[idx * c->k + t] = t < nu ? U[t].id : ORC_NONE;
            c->out_dist[idx * c->k + t] = t < nu ? U[t].d : INFINITY;
        }
    }
    ws_free(&ws);
    free(U);
}

/*
 * Stage 1 for the listed global ids `nodes` (all ids 0..N-1 when nodes is
 * NULL).  Xs is the matrix the beam scores (NULL: X).  Output row idx holds
 * the k-NN list of nodes[idx].  stats (nullable) receives {ndc, expansions}.
 * Returns 0, or -1 on bad arguments / malformed graphs.
 */
int oracle_cross_query(const float* X, const float* Xs, uint64_t ld, uint32_t dim,
                       int metric, const oracle_sub* subs, uint32_t h, uint32_t k,
                       uint32_t L, uint32_t rerank, const uint64_t* nodes,
                       uint64_t n_nodes, uint32_t* out_ids, float* out_dist,
                       int threads, uint64_t* stats, const uint8_t* valid)
{
    if (!X || !subs || h < 1 || k == 0 || L == 0 || dim == 0 || dim > 4096) return -1;
    for (uint32_t i = 0; i < h; ++i)
        if (!check_graph(subs[i].adj, subs[i].n, subs[i].stride, subs[i].entry)) return -1;
    if (threads < 1) threads = 1;
    uint64_t ndc[256] = {0}, ex[256] = {0};
    int err[256] = {0};
    cq_ctx c = {X, Xs ? Xs : X, ld, dim, metric, subs, h, k, L, rerank ? rerank : L,
                nodes, out_ids, out_dist, ndc, ex, err, valid};
    parallel_for(n_nodes, threads, cq_range, &c);
    uint64_t a = 0, bsum = 0;
    int bad = 0;
    for (int t = 0; t < 256; ++t) {
        a += ndc[t];
        bsum += ex[t];
        bad |= err[t];
    }
    if (stats) {
        stats[0] = a;
        stats[1] = bsum;
    }
    return bad ? -1 : 0;
}

/* Lower bound on L from the minimum querying strategy (Section 4.1.2):
 * ceil((k - min_u |C+(u)|) / (h - 1)), at least 1. */
uint32_t oracle_min_L(uint32_t k, uint32_t min_local, uint32_t h)
{
    if (h < 2) return 0;
    if (min_local >= k) return 1;
    uint32_t need = k - min_local;
    uint32_t l = (need + (h - 2)) / (h - 1);
    return l ? l : 1;
}

/* ------------------------------------------------------------------ */
/* Stage 2: k-NNG refinement (Algorithm 3) in synchronous rounds or in   */
/* streamlined micro-batches, with indegree repair (Algorithm 4) after   */
/* every round.                                                         */
/* ------------------------------------------------------------------ */

/*
 * Algorithm 4.  T(v) counts the lists that hold v.  Vertices with T = 0 are
 * taken in ascending id.  For such v*, its neighbours v are tried from the
 * closest; in N(v), from the farthest, the first entry v' that is not marked
 * replaced and has T(v') > 1 is evicted, and v* enters N(v) at its sorted
 * place (distance = the stored delta(v*, v)), flagged new and replaced.  A
 * list with a free slot takes v* without an eviction.  The outdegree never
 * grows past k.  Lists are N x k, sorted, NONE-padded.
 */
int oracle_repair(uint64_t N, uint32_t k, uint32_t* ids, float* dist,
                  uint8_t* flags, uint32_t* T, uint64_t* n_repaired)
{
    memset(T, 0, sizeof(uint32_t) * N);
    for (uint64_t i = 0; i < N * k; ++i) {
        if (ids[i] == ORC_NONE) continue;
        if (ids[i] >= N) return -1;
        T[ids[i]] += 1;
        flags[i] &= (uint8_t)~FLAG_REPLACED;
    }
    uint64_t fixed = 0;
    for (uint64_t vs = 0; vs < N; ++vs) {
        if (T[vs] != 0) continue;
        int done = 0;
        for (uint32_t s = 0; s < k && !done; ++s) {
            uint32_t v = ids[vs * k + s];
            if (v == ORC_NONE) break;
            float dnew = dist[vs * k + s];
            uint32_t* Lv = ids + (uint64_t)v * k;
            float* Dv = dist + (uint64_t)v * k;
            uint8_t* Fv = flags + (uint64_t)v * k;
            uint32_t cnt = 0;
            while (cnt < k && Lv[cnt] != ORC_NONE) ++cnt;
            int32_t drop = -1;
            if (cnt == k) {
                for (int32_t t = (int32_t)k - 1; t >= 0; --t) {
                    if (!(Fv[t] & FLAG_REPLACED) && T[Lv[t]] > 1) {
                        drop = t;
                        break;
                    }
                }
                if (drop < 0) continue;
                T[Lv[drop]] -= 1;
                for (uint32_t t = (uint32_t)drop; t + 1 < k; ++t) {
                    Lv[t] = Lv[t + 1];
                    Dv[t] = Dv[t + 1];
                    Fv[t] = Fv[t + 1];
                }
                Lv[k - 1] = ORC_NONE;
                Dv[k - 1] = INFINITY;
                Fv[k - 1] = 0;
                cnt = k - 1;
            }
            ent_t ins = {dnew, (uint32_t)vs, 0};
            uint32_t pos = 0;
            while (pos < cnt) {
                ent_t cur = {Dv[pos], Lv[pos], 0};
                if (ent_less(&ins, &cur)) break;
                ++pos;
            }
            for (uint32_t t = cnt; t > pos; --t) {
                Lv[t] = Lv[t - 1];
                Dv[t] = Dv[t - 1];
                Fv[t] = Fv[t - 1];
            }
            Lv[pos] = (uint32_t)vs;
            Dv[pos] = dnew;
            Fv[pos] = FLAG_NEW | FLAG_REPLACED;
            T[vs] += 1;
            ++fixed;
            done = 1;
        }
    }
    for (uint64_t i = 0; i < N * k; ++i) flags[i] &= (uint8_t)~FLAG_REPLACED;
    if (n_repaired) *n_repaired = fixed;
    return 0;
}

typedef struct {
    uint32_t a, b;
    float d;
} prop_t;

typedef struct {
    prop_t* v;
    size_t n, cap;
} prop_vec;

static int pv_push(prop_vec* pv, uint32_t a, uint32_t b, float d)
{
    if (pv->n == pv->cap) {
        size_t nc = pv->cap ? pv->cap * 2 : 1024;
        prop_t* nv = (prop_t*)realloc(pv->v, nc * sizeof(prop_t));
        if (!nv) return 0;
        pv->v = nv;
        pv->cap = nc;
    }
    pv->v[pv->n++] = (prop_t){a, b, d};
    return 1;
}

typedef struct {
    const float* X;
    uint64_t ld;
    uint32_t dim;
    int metric;
    const uint32_t* gsub;          /* sub-index of each global id */
    uint32_t k;
    const uint32_t* Sids;          /* snapshot lists */
    const float* Sdist;
    const uint64_t* cn_off;        /* CSR of Cn / Co per node */
    const uint32_t* cn;
    const uint64_t* co_off;
    const uint32_t* co;
    prop_vec* pv;                  /* per thread */
    int* err;
    uint64_t base;                 /* first vertex of the joined range */
} join_ctx;

/* worst key w[a] of the snapshot list of a (+inf when not full) */
static ent_t worst_of(const join_ctx* c, uint32_t a)
{
    uint64_t i = (uint64_t)a * c->k + c->k - 1;
    if (c->Sids[i] == ORC_NONE) return (ent_t){INFINITY, ORC_NONE, 0};
    return (ent_t){c->Sdist[i], c->Sids[i], 0};
}

static int propose(const join_ctx* c, prop_vec* pv, uint32_t a, uint32_t b)
{
    if (c->gsub[a] == c->gsub[b]) return 1;      /* pairs from different G_i only */
    float d = oracle_distance(c->X + (uint64_t)a * c->ld, c->X + (uint64_t)b * c->ld,
                              c->dim, c->metric);
    ent_t wa = worst_of(c, a), wb = worst_of(c, b);
    ent_t pa = {d, b, 0}, pb = {d, a, 0};
    if (ent_less(&pa, &wa) && !pv_push(pv, a, b, d)) return 0;
    if (ent_less(&pb, &wb) && !pv_push(pv, b, a, d)) return 0;
    return 1;
}

/* Update: every unordered pair of Cn(u), and every pair Cn(u) x Co(u),
 * whose ends come from different sub-indexes proposes each end to the
 * other (a proposal that cannot beat the target's current worst entry is
 * dropped here, which cannot change the apply step). */
static void join_range(void* p, uint64_t b, uint64_t e, int tid)
{
    join_ctx* c = (join_ctx*)p;
    prop_vec* pv = &c->pv[tid];
    for (uint64_t u = c->base + b; u < c->base + e; ++u) {
        const uint32_t* Cn = c->cn + c->cn_off[u];
        uint64_t nn = c->cn_off[u + 1] - c->cn_off[u];
        const uint32_t* Co = c->co + c->co_off[u];
        uint64_t no = c->co_off[u + 1] - c->co_off[u];
        for (uint64_t i = 0; i < nn; ++i) {
            for (uint64_t j = i + 1; j < nn; ++j)
                if (!propose(c, pv, Cn[i], Cn[j])) { c->err[tid] = 1; return; }
            for (uint64_t j = 0; j < no; ++j)
                if (!propose(c, pv, Cn[i], Co[j])) { c->err[tid] = 1; return; }
        }
    }
}

typedef struct {
    uint32_t k;
    uint32_t* ids;
    float* dist;
    uint8_t* flags;
    const uint32_t* Sids;
    const float* Sdist;
    const uint8_t* Sflags;
    const uint64_t* p_off;
    const prop_t* P;             /* proposals grouped by target a */
} apply_ctx;

/* list(a) <- first k of the (delta, id)-sorted union of the snapshot list
 * (entries keep their flags) and the proposals to a (entries are new); an
 * id that appears more than once keeps one entry, with the snapshot's flags
 * if it is in the snapshot. */
static void apply_range(void* p, uint64_t b, uint64_t e, int tid)
{
    (void)tid;
    apply_ctx* c = (apply_ctx*)p;
    size_t cap = 0;
    ent_t* U = NULL;
    for (uint64_t a = b; a < e; ++a) {
        uint64_t np = c->p_off[a + 1] - c->p_off[a];
        if (np == 0) continue;
        if (np + c->k > cap) {
            cap = np + c->k;
            free(U);
            U = (ent_t*)malloc(sizeof(ent_t) * cap);
        }
        size_t n = 0;
        for (uint32_t t = 0; t < c->k; ++t) {
            uint64_t i = a * c->k + t;
            if (c->Sids[i] == ORC_NONE) break;
            U[n++] = (ent_t){c->Sdist[i], c->Sids[i],
                             ENT_SNAPSHOT | (uint32_t)(c->Sflags[i] & (FLAG_NEW | FLAG_RNEW))};
        }
        for (uint64_t t = 0; t < np; ++t) {
            const prop_t* q = &c->P[c->p_off[a] + t];
            U[n++] = (ent_t){q->d, q->b, FLAG_NEW};
        }
        /* equal ids carry equal distances (delta is symmetric), so after the
         * sort the copies of an id are adjacent, in no particular order */
        qsort(U, n, sizeof(ent_t), ent_cmp);
        uint32_t outn = 0;
        for (size_t t = 0; t < n; ++t) {
            if (outn && c->ids[a * c->k + outn - 1] == U[t].id) {
                if (U[t].flag & ENT_SNAPSHOT)
                    c->flags[a * c->k + outn - 1] = (uint8_t)(U[t].flag & ~ENT_SNAPSHOT);
                continue;
            }
            if (outn == c->k) break;
            c->ids[a * c->k + outn] = U[t].id;
            c->dist[a * c->k + outn] = U[t].d;
            c->flags[a * c->k + outn] = (uint8_t)(U[t].flag & ~ENT_SNAPSHOT);
            ++outn;
        }
        for (; outn < c->k; ++outn) {
            c->ids[a * c->k + outn] = ORC_NONE;
            c->dist[a * c->k + outn] = INFINITY;
            c->flags[a * c->k + outn] = 0;
        }
    }
    free(U);
}

static int cmp_u32(const void* a, const void* b)
{
    uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

/* reverse lists: rev[v] = first k_rev by (stored delta, u) of {u : v in sel(u)},
 * where sel picks the list entries whose revnew mark matches want_new */
static int build_reverse(uint64_t N, uint32_t k, const uint32_t* ids, const float* dist,
                         const uint8_t* revnew, int want_new, uint32_t k_rev,
                         uint64_t* off /* N+1 */, uint32_t* out /* N*k_rev */)
{
    uint64_t* cnt = (uint64_t*)calloc(N + 1, sizeof(uint64_t));
    if (!cnt) return 0;
    for (uint64_t i = 0; i < N * k; ++i) {
        if (ids[i] == ORC_NONE) continue;
        if ((revnew[i] != 0) != (want_new != 0)) continue;
        cnt[ids[i] + 1] += 1;
    }
    for (uint64_t v = 0; v < N; ++v) cnt[v + 1] += cnt[v];
    ent_t* buf = (ent_t*)malloc(sizeof(ent_t) * (cnt[N] + 1));
    uint64_t* cur = (uint64_t*)malloc(sizeof(uint64_t) * (N + 1));
    if (!buf || !cur) { free(cnt); free(buf); free(cur); return 0; }
    memcpy(cur, cnt, sizeof(uint64_t) * (N + 1));
    for (uint64_t u = 0; u < N; ++u)
        for (uint32_t t = 0; t < k; ++t) {
            uint64_t i = u * k + t;
            if (ids[i] == ORC_NONE) continue;
            if ((revnew[i] != 0) != (want_new != 0)) continue;
            buf[cur[ids[i]]++] = (ent_t){dist[i], (uint32_t)u, 0};
        }
    off[0] = 0;
    for (uint64_t v = 0; v < N; ++v) {
        uint64_t n = cnt[v + 1] - cnt[v];
        qsort(buf + cnt[v], n, sizeof(ent_t), ent_cmp);
        if (n > k_rev) n = k_rev;
        for (uint64_t t = 0; t < n; ++t) out[off[v] + t] = buf[cnt[v] + t].id;
        off[v + 1] = off[v] + n;
    }
    free(cnt);
    free(buf);
    free(cur);
    return 1;
}

static int cmp_prop_target(const void* a, const void* b)
{
    const prop_t* x = (const prop_t*)a;
    const prop_t* y = (const prop_t*)b;
    if (x->a != y->a) return x->a < y->a ? -1 : 1;
    if (x->b != y->b) return x->b < y->b ? -1 : 1;
    return 0;
}

/*
 * Algorithm 3's Visit + Update for the vertices u in [lo, hi), on the lists
 * as they stand (a synchronous round is the range [0, N)):
 *  Visit: fwd_new(u)/fwd_old(u) split u's list by flag.  Each new entry of a
 *    visited list is recorded as a new reverse link of its target, and a
 *    visited vertex consumes the new reverse links recorded for it:
 *    rev_new(u) holds the w whose entry (w -> u) is such a link (recorded
 *    earlier, or by this range's Visit), rev_old(u) the w of u's other
 *    in-edges, each the first k_rev by (stored delta, w).  Cn(u) =
 *    fwd_new(u) U rev_new(u); Co(u) = (fwd_old(u) U rev_old(u)) \ Cn(u); then
 *    the new entries of u's list become old.  In a synchronous round every
 *    link is recorded and consumed in the same Visit.
 *  Update: see join_range; the proposals are applied to every list at once,
 *    before the next range is visited.
 * Returns the number of proposals applied, or -1 on failure.
 */
static int64_t refine_range(const float* X, uint64_t ld, uint32_t dim, int metric,
                            const uint32_t* gsub, uint64_t N, uint32_t k, uint32_t k_rev,
                            uint32_t* ids, float* dist, uint8_t* flags, int threads,
                            uint64_t lo, uint64_t hi)
{
    int64_t ret = -1;
    uint64_t *rn_off = NULL, *ro_off = NULL, *cn_off = NULL, *co_off = NULL, *p_off = NULL;
    uint32_t *rn = NULL, *ro = NULL, *cn = NULL, *co = NULL, *Sids = NULL;
    float* Sdist = NULL;
    uint8_t* Sflags = NULL;
    uint8_t* revnew = NULL;
    prop_vec pv[256];
    int err[256] = {0};
    memset(pv, 0, sizeof(pv));
    prop_t* P = NULL;
    uint32_t* tmp = NULL;

    rn_off = (uint64_t*)malloc(sizeof(uint64_t) * (N + 1));
    ro_off = (uint64_t*)malloc(sizeof(uint64_t) * (N + 1));
    rn = (uint32_t*)malloc(sizeof(uint32_t) * (N * k_rev + 1));
    ro = (uint32_t*)malloc(sizeof(uint32_t) * (N * k_rev + 1));
    cn_off = (uint64_t*)malloc(sizeof(uint64_t) * (N + 1));
    co_off = (uint64_t*)malloc(sizeof(uint64_t) * (N + 1));
    cn = (uint32_t*)malloc(sizeof(uint32_t) * (N * (k + k_rev) + 1));
    co = (uint32_t*)malloc(sizeof(uint32_t) * (N * (k + k_rev) + 1));
    tmp = (uint32_t*)malloc(sizeof(uint32_t) * (2 * ((size_t)k + k_rev) + 1));
    Sids = (uint32_t*)malloc(sizeof(uint32_t) * N * k);
    Sdist = (float*)malloc(sizeof(float) * N * k);
    Sflags = (uint8_t*)malloc(N * k + 1);
    if (!rn_off || !ro_off || !rn || !ro || !cn_off || !co_off || !cn || !co || !tmp ||
        !Sids || !Sdist || !Sflags)
        goto done;
    revnew = (uint8_t*)malloc(N * k + 1);
    if (!revnew) goto done;
    for (uint64_t i = 0; i < N * k; ++i) {
        uint64_t o = i / k;
        revnew[i] = (flags[i] & FLAG_RNEW) || (o >= lo && o < hi && (flags[i] & FLAG_NEW));
    }
    if (!build_reverse(N, k, ids, dist, revnew, 1, k_rev, rn_off, rn)) goto done;
    if (!build_reverse(N, k, ids, dist, revnew, 0, k_rev, ro_off, ro)) goto done;

    cn_off[0] = co_off[0] = 0;
    for (uint64_t u = 0; u < N; ++u) {
        if (u < lo || u >= hi) {           /* not visited in this range */
            cn_off[u + 1] = cn_off[u];
            co_off[u + 1] = co_off[u];
            continue;
        }
        /* Cn(u): sorted unique ids of fwd_new(u) U rev_new(u) */
        size_t n = 0;
        for (uint32_t t = 0; t < k; ++t) {
            uint64_t i = u * k + t;
            if (ids[i] != ORC_NONE && (flags[i] & FLAG_NEW)) tmp[n++] = ids[i];
        }
        for (uint64_t t = rn_off[u]; t < rn_off[u + 1]; ++t) tmp[n++] = rn[t];
        qsort(tmp, n, sizeof(uint32_t), cmp_u32);
        uint64_t w = cn_off[u];
        for (size_t t = 0; t < n; ++t)
            if (t == 0 || tmp[t] != tmp[t - 1]) cn[w++] = tmp[t];
        cn_off[u + 1] = w;
        /* Co(u): sorted unique ids of fwd_old(u) U rev_old(u), minus Cn(u) */
        n = 0;
        for (uint32_t t = 0; t < k; ++t) {
            uint64_t i = u * k + t;
            if (ids[i] != ORC_NONE && !(flags[i] & FLAG_NEW)) tmp[n++] = ids[i];
        }
        for (uint64_t t = ro_off[u]; t < ro_off[u + 1]; ++t) tmp[n++] = ro[t];
        qsort(tmp, n, sizeof(uint32_t), cmp_u32);
        uint64_t wo = co_off[u];
        for (size_t t = 0; t < n; ++t) {
            if (t > 0 && tmp[t] == tmp[t - 1]) continue;
            int in_cn = 0;
            for (uint64_t q = cn_off[u]; q < cn_off[u + 1]; ++q)
                if (cn[q] == tmp[t]) { in_cn = 1; break; }
            if (!in_cn) co[wo++] = tmp[t];
        }
        co_off[u + 1] = wo;
    }
    /* reverse links: consumed by a visited target, recorded for a later one */
    for (uint64_t i = 0; i < N * k; ++i) {
        if (ids[i] == ORC_NONE) continue;
        uint64_t o = i / k;
        if (ids[i] >= lo && ids[i] < hi) flags[i] &= (uint8_t)~FLAG_RNEW;
        else if (o >= lo && o < hi && (flags[i] & FLAG_NEW)) flags[i] |= (uint8_t)FLAG_RNEW;
    }
    for (uint64_t i = lo * k; i < hi * k; ++i) flags[i] &= (uint8_t)~FLAG_NEW;
    memcpy(Sids, ids, sizeof(uint32_t) * N * k);
    memcpy(Sdist, dist, sizeof(float) * N * k);
    memcpy(Sflags, flags, N * k);

    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    join_ctx jc = {X, ld, dim, metric, gsub, k, Sids, Sdist, cn_off, cn, co_off, co, pv, err, lo};
    parallel_for(hi - lo, threads, join_range, &jc);
    size_t total = 0;
    for (int t = 0; t < 256; ++t) {
        if (err[t]) goto done;
        total += pv[t].n;
    }
    P = (prop_t*)malloc(sizeof(prop_t) * (total + 1));
    p_off = (uint64_t*)calloc(N + 1, sizeof(uint64_t));
    if (!P || !p_off) goto done;
    size_t w = 0;
    for (int t = 0; t < 256; ++t) {
        if (pv[t].n) memcpy(P + w, pv[t].v, pv[t].n * sizeof(prop_t));
        w += pv[t].n;
    }
    qsort(P, total, sizeof(prop_t), cmp_prop_target);
    for (size_t t = 0; t < total; ++t) p_off[P[t].a + 1] += 1;
    for (uint64_t a = 0; a < N; ++a) p_off[a + 1] += p_off[a];
    apply_ctx ac = {k, ids, dist, flags, Sids, Sdist, Sflags, p_off, P};
    parallel_for(N, threads, apply_range, &ac);
    ret = (int64_t)total;
done:
    for (int t = 0; t < 256; ++t) free(pv[t].v);
    free(rn_off); free(ro_off); free(rn); free(ro); free(cn_off); free(co_off);
    free(cn); free(co); free(tmp); free(Sids); free(Sdist); free(Sflags); free(revnew); free(P);
    free(p_off);
    return ret;
}

/*
 * Stage 2 on an N x k list set sorted by (delta, id).  `flags` (N x k, bit 0 =
 * new, bit 2 = an unconsumed new reverse link, FLAG_RNEW) is in/out; pass
 * all-new flags for a stage-1 output.  Synchronous rounds never leave
 * FLAG_RNEW set.  Runs exactly
 * `rounds` rounds; after each, indegree repair when do_repair != 0.  T (N)
 * receives the indegrees after the last round.  stats (nullable) receives
 * {proposals, repaired}.
 *
 * batches <= 1: each round visits every vertex against one snapshot
 * (synchronous).  batches = B > 1: the streamlined form of Section 4.2.1,
 * in which a vertex's Visit and Update read the latest graph: each round
 * visits the ranges [b N / B, (b + 1) N / B), b = 0 .. B-1, in turn, and a
 * range's proposals are applied before the next range is visited.  B = N
 * is the one-vertex-at-a-time pass, in ascending id.
 */
int oracle_refine(const float* X, uint64_t ld, uint32_t dim, int metric,
                  const oracle_sub* subs, uint32_t h, uint64_t N, uint32_t k,
                  uint32_t rounds, uint32_t k_rev, uint32_t* ids, float* dist,
                  uint8_t* flags, uint32_t* T, int do_repair, int threads,
                  uint64_t* stats, uint32_t batches)
{
    if (!X || !ids || !dist || !flags || !T || k == 0) return -1;
    if (k_rev == 0) k_rev = k;
    uint32_t* gsub = (uint32_t*)malloc(sizeof(uint32_t) * (N + 1));
    if (!gsub) return -1;
    for (uint64_t v = 0; v < N; ++v) {
        gsub[v] = sub_of(subs, h, v);
        if (gsub[v] >= h) { free(gsub); return -1; }
    }
    uint64_t props = 0, rep = 0;
    if (batches < 1) batches = 1;
    for (uint32_t r = 0; r < rounds; ++r) {
        for (uint32_t bt = 0; bt < batches; ++bt) {
            uint64_t lo = N * bt / batches, hi = N * (bt + 1) / batches;
            if (lo == hi) continue;
            int64_t p = refine_range(X, ld, dim, metric, gsub, N, k, k_rev, ids, dist, flags,
                                     threads, lo, hi);
            if (p < 0) { free(gsub); return -1; }
            props += (uint64_t)p;
        }
        if (do_repair) {
            uint64_t nr = 0;
            if (oracle_repair(N, k, ids, dist, flags, T, &nr)) { free(gsub); return -1; }
            rep += nr;
        }
    }
    /* T for the prune: the indegrees of the final lists */
    memset(T, 0, sizeof(uint32_t) * N);
    for (uint64_t i = 0; i < N * k; ++i)
        if (ids[i] != ORC_NONE) T[ids[i]] += 1;
    if (stats) {
        stats[0] = props;
        stats[1] = rep;
    }
    free(gsub);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Stage 3: k-NNG -> PG (Algorithm 5).                                  */
/* ------------------------------------------------------------------ */

typedef struct {
    const float* X;
    uint64_t ld;
    uint32_t dim;
    int metric;
    uint32_t k, R;
    const uint32_t* ids;
    const float* dist;
    const uint32_t* T;
    uint32_t* sel_ids;     /* N x R */
    float* sel_dist;
    uint32_t* sel_n;
    int rule;              /* ORC_SEL_* */
    float param;           /* alpha or tau */
} prune_ctx;

/* The Euclidean distance behind delta: sqrt(delta) for squared L2, and
 * sqrt(2 delta) for cosine on unit vectors (|a - b|^2 = 2 (1 - <a,b>)),
 * with a negative rounding residue read as 0.  sqrtf is correctly rounded. */
static float euclid_of(float d, int metric)
{
    float s = metric == ORC_COS ? 2.0f * d : d;
    return sqrtf(s > 0.0f ? s : 0.0f);
}

/*
 * Whether an already kept neighbour w, at delta(w, v) = dwv, leaves the
 * candidate v, at delta(u, v) = duv, selectable (Section 4.3.1 names RNG
 * and, as swap-ins, alpha-RNG and tau-MNG):
 *  - RNG (Algorithm 5): duv < dwv.
 *  - alpha-RNG: v survives w when |u - v| < alpha |w - v| (Vamana's robust
 *    prune); on delta, which is the squared distance for L2 and half of it
 *    for cosine, that is duv < alpha^2 dwv, with alpha^2 rounded to FP32
 *    once and the product rounded once.
 *  - tau-MNG: w occludes v when |w - v| < |u - v| - 3 tau (the
 *    tau-monotonic graph's edge rule); v survives when
 *    e(duv) < e(dwv) + 3 tau on the Euclidean distances e, strict as in
 *    Algorithm 5, with 3 tau rounded to FP32 once.
 */
static int pair_keeps(const prune_ctx* c, float duv, float dwv)
{
    if (c->rule == ORC_SEL_ALPHA) {
        float a2 = c->param * c->param;
        float lim = a2 * dwv;
        return duv < lim;
    }
    if (c->rule == ORC_SEL_TAU) {
        float t = 3.0f * c->param;
        float lim = euclid_of(dwv, c->metric) + t;
        return euclid_of(duv, c->metric) < lim;
    }
    return duv < dwv;
}

/* Neighbour selection of vertex u: scan N(u) from the closest; keep v when
 * T(v) = 1 or every kept w leaves v selectable (pair_keeps; Algorithm 5's
 * rule is delta(u, v) < delta(w, v)); stop at R kept.  Writes the kept ids /
 * distances to out_ids / out_dist (R slots) and returns their number. */
static uint32_t select_one(const prune_ctx* c, uint64_t u, uint32_t* out_ids, float* out_dist)
{
    uint32_t ns = 0;
    for (uint32_t s = 0; s < c->k && ns < c->R; ++s) {
        uint32_t v = c->ids[u * c->k + s];
        if (v == ORC_NONE) break;
        float duv = c->dist[u * c->k + s];
        int keep = c->T && c->T[v] == 1;   /* no indegree recorder: no exemption */
        if (!keep) {
            keep = 1;
            for (uint32_t q = 0; q < ns; ++q) {
                uint32_t w = out_ids[q];
                float dwv = oracle_distance(c->X + (uint64_t)w * c->ld,
                                            c->X + (uint64_t)v * c->ld, c->dim, c->metric);
                if (!pair_keeps(c, duv, dwv)) { keep = 0; break; }
            }
        }
        if (keep) {
            out_ids[ns] = v;
            out_dist[ns] = duv;
            ++ns;
        }
    }
    return ns;
}

static void select_range(void* p, uint64_t b, uint64_t e, int tid)
{
    (void)tid;
    prune_ctx* c = (prune_ctx*)p;
    for (uint64_t u = b; u < e; ++u)
        c->sel_n[u] = select_one(c, u, c->sel_ids + u * c->R, c->sel_dist + u * c->R);
}

/*
 * Neighbour selection, then connectivity enhancement on the selected edge
 * set E' taken as a whole: N(u) <- first R of the (delta, id)-sorted,
 * id-unique union of u's selected neighbours and {v : u selected by v}.
 * Writes out_ids (N x R, NONE padded), out_dist (nullable) and out_deg.
 */
static int rule_ok(int rule, float param, int metric)
{
    if (rule == ORC_SEL_RNG) return 1;
    if (metric == ORC_IP) return 0;   /* not a metric: transform MIPS to L2 first */
    if (rule == ORC_SEL_ALPHA) return param >= 1.0f;
    if (rule == ORC_SEL_TAU) return param >= 0.0f;
    return 0;
}

int oracle_prune(const float* X, uint64_t ld, uint32_t dim, int metric, uint64_t N,
                 uint32_t k, const uint32_t* ids, const float* dist, const uint32_t* T,
                 uint32_t R, uint32_t* out_ids, float* out_dist, uint32_t* out_deg,
                 int threads, int rule, float param)
{
    if (!X || !ids || !dist || !T || !out_ids || !out_deg || R == 0 || k == 0) return -1;
    if (!rule_ok(rule, param, metric)) return -1;
    for (uint64_t i = 0; i < N * k; ++i)
        if (ids[i] != ORC_NONE && ids[i] >= N) return -1;
    uint32_t* sel_ids = (uint32_t*)malloc(sizeof(uint32_t) * N * R);
    float* sel_dist = (float*)malloc(sizeof(float) * N * R);
    uint32_t* sel_n = (uint32_t*)malloc(sizeof(uint32_t) * N);
    uint64_t* roff = (uint64_t*)calloc(N + 1, sizeof(uint64_t));
    if (!sel_ids || !sel_dist || !sel_n || !roff) {
        free(sel_ids); free(sel_dist); free(sel_n); free(roff);
        return -1;
    }
    prune_ctx c = {X, ld, dim, metric, k, R, ids, dist, T, sel_ids, sel_dist, sel_n, rule, param};
    parallel_for(N, threads, select_range, &c);

    for (uint64_t u = 0; u < N; ++u)
        for (uint32_t q = 0; q < sel_n[u]; ++q) roff[sel_ids[u * R + q] + 1] += 1;
    for (uint64_t v = 0; v < N; ++v) roff[v + 1] += roff[v];
    ent_t* rev = (ent_t*)malloc(sizeof(ent_t) * (roff[N] + 1));
    uint64_t* cur = (uint64_t*)malloc(sizeof(uint64_t) * (N + 1));
    ent_t* U = (ent_t*)malloc(sizeof(ent_t) * ((size_t)R + 1));
    if (!rev || !cur || !U) {
        free(sel_ids); free(sel_dist); free(sel_n); free(roff); free(rev); free(cur); free(U);
        return -1;
    }
    memcpy(cur, roff, sizeof(uint64_t) * (N + 1));
    for (uint64_t u = 0; u < N; ++u)
        for (uint32_t q = 0; q < sel_n[u]; ++q) {
            uint32_t v = sel_ids[u * R + q];
            rev[cur[v]++] = (ent_t){sel_dist[u * R + q], (uint32_t)u, 0};
        }
    size_t ucap = R + 1;
    for (uint64_t u = 0; u < N; ++u) {
        size_t n = sel_n[u] + (roff[u + 1] - roff[u]);
        if (n > ucap) {
            ucap = n;
            free(U);
            U = (ent_t*)malloc(sizeof(ent_t) * ucap);
            if (!U) break;
        }
        size_t m = 0;
        for (uint32_t q = 0; q < sel_n[u]; ++q)
            U[m++] = (ent_t){sel_dist[u * R + q], sel_ids[u * R + q], 0};
        for (uint64_t t = roff[u]; t < roff[u + 1]; ++t) U[m++] = rev[t];
        qsort(U, m, sizeof(ent_t), ent_cmp);
        uint32_t o = 0;
        for (size_t t = 0; t < m && o < R; ++t) {
            if (o && out_ids[u * R + o - 1] == U[t].id) continue;
            out_ids[u * R + o] = U[t].id;
            if (out_dist) out_dist[u * R + o] = U[t].d;
            ++o;
        }
        out_deg[u] = o;
        for (; o < R; ++o) {
            out_ids[u * R + o] = ORC_NONE;
            if (out_dist) out_dist[u * R + o] = INFINITY;
        }
    }
    int ok = U != NULL;
    free(sel_ids); free(sel_dist); free(sel_n); free(roff); free(rev); free(cur); free(U);
    return ok ? 0 : -1;
}

/* Stage 3 for the listed vertices only, on the full N x k lists: row r of
 * out_ids / out_dist / out_deg is what oracle_prune writes for vertex
 * rows[r].  Each listed u takes its own selection and the reverse of every
 * selection that picks u; the vertices that can pick u are those whose list
 * holds u, found through an inverted index of the lists.  Selections are
 * computed for u and those vertices only, so a sample of a large graph costs
 * a few selections per listed vertex. */
typedef struct {
    const prune_ctx* c;
    const uint64_t* rows;
    const uint64_t* in_off;   /* inverted index: lists holding v */
    const uint32_t* in_src;
    uint32_t* out_ids;
    float* out_dist;
    uint32_t* out_deg;
    int* err;
} prune_rows_ctx;

static void prune_rows_range(void* p, uint64_t b, uint64_t e, int tid)
{
    prune_rows_ctx* r = (prune_rows_ctx*)p;
    const prune_ctx* c = r->c;
    uint32_t R = c->R;
    uint32_t* sid = (uint32_t*)malloc(sizeof(uint32_t) * ((size_t)R + 1));
    float* sdd = (float*)malloc(sizeof(float) * ((size_t)R + 1));
    size_t ucap = 0;
    ent_t* U = NULL;
    if (!sid || !sdd) { r->err[tid] = 1; free(sid); free(sdd); return; }
    for (uint64_t idx = b; idx < e; ++idx) {
        uint64_t u = r->rows[idx];
        uint64_t nin = r->in_off[u + 1] - r->in_off[u];
        if (R + nin + 1 > ucap) {
            ucap = R + nin + 1;
            free(U);
            U = (ent_t*)malloc(sizeof(ent_t) * ucap);
            if (!U) { r->err[tid] = 1; break; }
        }
        size_t m = 0;
        uint32_t ns = select_one(c, u, sid, sdd);
        for (uint32_t q = 0; q < ns; ++q) U[m++] = (ent_t){sdd[q], sid[q], 0};
        for (uint64_t t = r->in_off[u]; t < r->in_off[u + 1]; ++t) {
            uint32_t v = r->in_src[t];
            uint32_t nv = select_one(c, v, sid, sdd);
            for (uint32_t q = 0; q < nv; ++q)
                if (sid[q] == (uint32_t)u) U[m++] = (ent_t){sdd[q], v, 0};
        }
        qsort(U, m, sizeof(ent_t), ent_cmp);
        uint32_t o = 0;
        for (size_t t = 0; t < m && o < R; ++t) {
            if (o && r->out_ids[idx * R + o - 1] == U[t].id) continue;
            r->out_ids[idx * R + o] = U[t].id;
            r->out_dist[idx * R + o] = U[t].d;
            ++o;
        }
        r->out_deg[idx] = o;
        for (; o < R; ++o) {
            r->out_ids[idx * R + o] = ORC_NONE;
            r->out_dist[idx * R + o] = INFINITY;
        }
    }
    free(sid);
    free(sdd);
    free(U);
}

int oracle_prune_rows(const float* X, uint64_t ld, uint32_t dim, int metric, uint64_t N,
                      uint32_t k, const uint32_t* ids, const float* dist, const uint32_t* T,
                      uint32_t R, const uint64_t* rows, uint64_t nrows, uint32_t* out_ids,
                      float* out_dist, uint32_t* out_deg, int threads, int rule, float param)
{
    if (!X || !ids || !dist || !T || !rows || !out_ids || !out_dist || !out_deg || R == 0 ||
        k == 0)
        return -1;
    if (!rule_ok(rule, param, metric)) return -1;
    for (uint64_t i = 0; i < N * k; ++i)
        if (ids[i] != ORC_NONE && ids[i] >= N) return -1;
    for (uint64_t i = 0; i < nrows; ++i)
        if (rows[i] >= N) return -1;
    uint64_t* in_off = (uint64_t*)calloc(N + 2, sizeof(uint64_t));
    uint64_t* cur = (uint64_t*)malloc(sizeof(uint64_t) * (N + 1));
    uint32_t* in_src = (uint32_t*)malloc(sizeof(uint32_t) * (N * k + 1));
    if (!in_off || !cur || !in_src) { free(in_off); free(cur); free(in_src); return -1; }
    for (uint64_t i = 0; i < N * k; ++i)
        if (ids[i] != ORC_NONE) in_off[ids[i] + 1] += 1;
    for (uint64_t v = 0; v < N; ++v) in_off[v + 1] += in_off[v];
    memcpy(cur, in_off, sizeof(uint64_t) * (N + 1));
    for (uint64_t u = 0; u < N; ++u)
        for (uint32_t t = 0; t < k; ++t) {
            uint32_t v = ids[u * k + t];
            if (v != ORC_NONE) in_src[cur[v]++] = (uint32_t)u;
        }
    prune_ctx c = {X, ld, dim, metric, k, R, ids, dist, T, NULL, NULL, NULL, rule, param};
    int err[256] = {0};
    prune_rows_ctx rc = {&c, rows, in_off, in_src, out_ids, out_dist, out_deg, err};
    parallel_for(nrows, threads, prune_rows_range, &rc);
    int bad = 0;
    for (int t = 0; t < 256; ++t) bad |= err[t];
    free(in_off);
    free(cur);
    free(in_src);
    return bad ? -1 : 0;
}

/* Entry of the merged graph: the entry point of the largest sub-index
 * (lowest index on ties), mapped to its global id.  With validity flags
 * (nullable): when that entry is invalid, the smallest valid global id of
 * the same sub-index; sub-indexes without a valid vertex are passed over
 * (next largest, lowest index on ties); ORC_NONE when no vertex is valid. */
uint64_t oracle_merged_entry(const oracle_sub* subs, uint32_t h, const uint8_t* valid)
{
    uint8_t* used = (uint8_t*)calloc(h ? h : 1, 1);
    uint64_t out = ORC_NONE;
    for (uint32_t round = 0; round < h && used; ++round) {
        uint32_t best = h;
        for (uint32_t i = 0; i < h; ++i)
            if (!used[i] && (best == h || subs[i].n > subs[best].n)) best = i;
        used[best] = 1;
        uint64_t e = subs[best].off + subs[best].entry;
        if (!valid || valid[e]) { out = e; break; }
        for (uint64_t g = subs[best].off; g < subs[best].off + subs[best].n; ++g)
            if (valid[g]) { out = g; break; }
        if (out != ORC_NONE) break;
    }
    free(used);
    return out;
}

/* All three stages.  out_ids N x R, out_deg N, *entry. */
int oracle_merge(const float* X, uint64_t ld, uint32_t dim, int metric,
                 const oracle_sub* subs, uint32_t h, uint32_t k, uint32_t L,
                 uint32_t rounds, uint32_t k_rev, uint32_t R, uint32_t* out_ids,
                 uint32_t* out_deg, uint64_t* entry, int threads, const uint8_t* valid,
                 uint32_t batches)
{
    uint64_t N = 0;
    for (uint32_t i = 0; i < h; ++i) N += subs[i].n;
    uint32_t* ids = (uint32_t*)malloc(sizeof(uint32_t) * N * k);
    float* dist = (float*)malloc(sizeof(float) * N * k);
    uint8_t* flags = (uint8_t*)malloc(N * k);
    uint32_t* T = (uint32_t*)malloc(sizeof(uint32_t) * N);
    int rc = -1;
    if (!ids || !dist || !flags || !T) goto out;
    if (oracle_cross_query(X, NULL, ld, dim, metric, subs, h, k, L, 0, NULL, N, ids, dist,
                           threads, NULL, valid))
        goto out;
    for (uint64_t i = 0; i < N * k; ++i) flags[i] = ids[i] == ORC_NONE ? 0 : FLAG_NEW;
    if (oracle_refine(X, ld, dim, metric, subs, h, N, k, rounds, k_rev, ids, dist, flags, T,
                      1, threads, NULL, batches))
        goto out;
    if (oracle_prune(X, ld, dim, metric, N, k, ids, dist, T, R, out_ids, NULL, out_deg,
                     threads, ORC_SEL_RNG, 0.0f))
        goto out;
    *entry = oracle_merged_entry(subs, h, valid);
    rc = 0;
out:
    free(ids); free(dist); free(flags); free(T);
    return rc;
}

/* ------------------------------------------------------------------ */
/* HNSW-adaptive merging (Section 4.3.3): upper layers over the merged  */
/* base graph.                                                          */
/* ------------------------------------------------------------------ */

/*
 * level[v] (drawn by the caller from HNSW's level distribution) puts v in
 * layers 1..level[v]; layer 0 is the merged graph itself.  Each layer
 * l = 1..max_level with members V_l (ascending ids) is built in four steps:
 *   cand(u)  the ef nearest other members of V_l by (delta, id) (exact)
 *   sel(u)   HNSW's neighbour heuristic (the RNG rule of Algorithm 5, with
 *            no indegree exemption) over cand(u), up to M
 *   uni(u)   the first 2M of the (delta, id)-sorted, id-unique union of
 *            sel(u) and {v in V_l : u in sel(v)} (bidirectional edges)
 *   adj(u)   the heuristic again over uni(u), up to M (HNSW's pruning of the
 *            neighbours that gained an edge)
 * Outputs, layers concatenated in order l = 1..max_level: layer_ids (the
 * members), layer_adj (M per member, global ids, ORC_NONE padded),
 * layer_count[l - 1] = |V_l|.  *top = the smallest id of the highest
 * non-empty layer (ORC_NONE when every layer is empty).
 */
int oracle_hnsw_layers(const float* X, uint64_t ld, uint32_t dim, int metric, uint64_t N,
                       const uint8_t* level, uint32_t max_level, uint32_t M, uint32_t ef,
                       uint32_t* layer_ids, uint32_t* layer_adj, uint64_t* layer_count,
                       uint32_t* top, int threads)
{
    if (!X || !level || !layer_ids || !layer_adj || !layer_count || !top || M == 0 || ef == 0)
        return -1;
    uint32_t* cid = (uint32_t*)malloc(sizeof(uint32_t) * (N * ef + 1));
    float* cdd = (float*)malloc(sizeof(float) * (N * ef + 1));
    uint32_t* uid = (uint32_t*)malloc(sizeof(uint32_t) * (N * 2 * M + 1));
    float* udd = (float*)malloc(sizeof(float) * (N * 2 * M + 1));
    uint32_t* deg = (uint32_t*)malloc(sizeof(uint32_t) * (N + 1));
    uint32_t* adj = (uint32_t*)malloc(sizeof(uint32_t) * (N * M + 1));
    uint32_t* mem = (uint32_t*)malloc(sizeof(uint32_t) * (N + 1));
    ent_t* buf = (ent_t*)malloc(sizeof(ent_t) * (N + 1));
    int rc = -1;
    if (!cid || !cdd || !uid || !udd || !deg || !adj || !mem || !buf) goto out;
    *top = ORC_NONE;
    uint64_t outrow = 0;
    for (uint32_t l = 1; l <= max_level; ++l) {
        uint64_t n = 0;
        for (uint64_t v = 0; v < N; ++v)
            if (level[v] >= l) mem[n++] = (uint32_t)v;
        layer_count[l - 1] = n;
        if (n) *top = mem[0];
        /* candidates: lists indexed by global id, empty for non-members */
        for (uint64_t i = 0; i < N * ef; ++i) { cid[i] = ORC_NONE; cdd[i] = INFINITY; }
        for (uint64_t a = 0; a < n; ++a) {
            uint32_t u = mem[a];
            uint64_t m = 0;
            for (uint64_t b = 0; b < n; ++b) {
                if (b == a) continue;
                buf[m++] = (ent_t){oracle_distance(X + (uint64_t)u * ld, X + (uint64_t)mem[b] * ld,
                                                   dim, metric), mem[b], 0};
            }
            qsort(buf, m, sizeof(ent_t), ent_cmp);
            for (uint64_t t = 0; t < m && t < ef; ++t) {
                cid[(uint64_t)u * ef + t] = buf[t].id;
                cdd[(uint64_t)u * ef + t] = buf[t].d;
            }
        }
        /* sel(u): the heuristic over cand(u), up to M */
        prune_ctx c1 = {X, ld, dim, metric, ef, M, cid, cdd, NULL, NULL, NULL, NULL,
                        ORC_SEL_RNG, 0.0f};
        uint32_t* sid = adj;            /* N x M selections (members' rows) */
        float* sdd = (float*)malloc(sizeof(float) * (N * M + 1));
        uint32_t* sn = deg;
        uint64_t* roff = (uint64_t*)calloc(N + 1, sizeof(uint64_t));
        if (!sdd || !roff) { free(sdd); free(roff); goto out; }
        for (uint64_t v = 0; v < N; ++v) sn[v] = 0;
        for (uint64_t a2 = 0; a2 < n; ++a2) {
            uint32_t u = mem[a2];
            sn[u] = select_one(&c1, u, sid + (uint64_t)u * M, sdd + (uint64_t)u * M);
        }
        /* uni(u): sel(u) and the reverse of every selection that picks u */
        for (uint64_t a2 = 0; a2 < n; ++a2) {
            uint32_t u = mem[a2];
            for (uint32_t t = 0; t < sn[u]; ++t) roff[sid[(uint64_t)u * M + t] + 1] += 1;
        }
        for (uint64_t v = 0; v < N; ++v) roff[v + 1] += roff[v];
        ent_t* rev = (ent_t*)malloc(sizeof(ent_t) * (roff[N] + 1));
        uint64_t* cur = (uint64_t*)malloc(sizeof(uint64_t) * (N + 1));
        ent_t* U = (ent_t*)malloc(sizeof(ent_t) * (M + roff[N] + 1));
        if (!rev || !cur || !U) { free(sdd); free(roff); free(rev); free(cur); free(U); goto out; }
        memcpy(cur, roff, sizeof(uint64_t) * (N + 1));
        for (uint64_t a2 = 0; a2 < n; ++a2) {
            uint32_t u = mem[a2];
            for (uint32_t t = 0; t < sn[u]; ++t) {
                uint32_t v = sid[(uint64_t)u * M + t];
                rev[cur[v]++] = (ent_t){sdd[(uint64_t)u * M + t], u, 0};
            }
        }
        for (uint64_t i = 0; i < N * 2 * M; ++i) { uid[i] = ORC_NONE; udd[i] = INFINITY; }
        for (uint64_t a2 = 0; a2 < n; ++a2) {
            uint32_t u = mem[a2];
            size_t m = 0;
            for (uint32_t t = 0; t < sn[u]; ++t)
                U[m++] = (ent_t){sdd[(uint64_t)u * M + t], sid[(uint64_t)u * M + t], 0};
            for (uint64_t t = roff[u]; t < roff[u + 1]; ++t) U[m++] = rev[t];
            qsort(U, m, sizeof(ent_t), ent_cmp);
            uint32_t o = 0;
            for (size_t t = 0; t < m && o < 2 * M; ++t) {
                if (o && uid[(uint64_t)u * 2 * M + o - 1] == U[t].id) continue;
                uid[(uint64_t)u * 2 * M + o] = U[t].id;
                udd[(uint64_t)u * 2 * M + o] = U[t].d;
                ++o;
            }
        }
        free(rev); free(cur); free(U); free(roff);
        /* adj(u): the heuristic again over uni(u), up to M */
        prune_ctx c2 = {X, ld, dim, metric, 2 * M, M, uid, udd, NULL, NULL, NULL, NULL,
                        ORC_SEL_RNG, 0.0f};
        for (uint64_t a2 = 0; a2 < n; ++a2) {
            uint32_t u = mem[a2];
            uint32_t* row = layer_adj + (outrow + a2) * M;
            uint32_t ns = select_one(&c2, u, row, sdd);
            for (uint32_t t = ns; t < M; ++t) row[t] = ORC_NONE;
            layer_ids[outrow + a2] = u;
        }
        free(sdd);
        outrow += n;
    }
    rc = 0;
out:
    free(cid); free(cdd); free(uid); free(udd); free(deg); free(adj); free(mem); free(buf);
    return rc;
}

/*
 * Search over the hierarchy: from `top`, greedy descent through layers
 * max_level..1 (move to the closest neighbour in the layer while it is
 * closer than the current vertex, ties by id), then Algorithm 1 on the base
 * graph from the vertex reached.  Rows of layer l are found by binary search
 * of the member ids.  Returns the pool size written to out_ids / out_dist.
 */
int oracle_hnsw_search(const float* q, const float* X, uint64_t ld, uint32_t dim, int metric,
                       uint64_t N, const uint32_t* base_adj, uint32_t stride,
                       const uint32_t* layer_ids, const uint32_t* layer_adj,
                       const uint64_t* layer_count, uint32_t max_level, uint32_t M,
                       uint32_t top, uint32_t L, uint32_t* out_ids, float* out_dist)
{
    if (top == ORC_NONE || top >= N || L == 0) return -1;
    uint64_t start[256];
    uint64_t acc = 0;
    if (max_level > 255) return -1;
    for (uint32_t l = 1; l <= max_level; ++l) { start[l] = acc; acc += layer_count[l - 1]; }
    uint32_t cur = top;
    ent_t best = {oracle_distance(q, X + (uint64_t)cur * ld, dim, metric), cur, 0};
    for (uint32_t l = max_level; l >= 1; --l) {
        uint64_t n = layer_count[l - 1];
        if (n == 0) continue;
        for (;;) {
            uint64_t lo = 0, hi = n;
            const uint32_t* ids = layer_ids + start[l];
            while (lo < hi) {
                uint64_t mid = (lo + hi) / 2;
                if (ids[mid] < best.id) lo = mid + 1; else hi = mid;
            }
            if (lo >= n || ids[lo] != best.id) break;   /* not a member: stay */
            const uint32_t* row = layer_adj + (start[l] + lo) * M;
            ent_t nb = best;
            for (uint32_t t = 0; t < M; ++t) {
                if (row[t] == ORC_NONE) continue;
                ent_t e = {oracle_distance(q, X + (uint64_t)row[t] * ld, dim, metric), row[t], 0};
                if (ent_less(&e, &nb)) nb = e;
            }
            if (nb.id == best.id) break;
            best = nb;
        }
    }
    uint64_t ndc = 0, nexp = 0;
    int n = oracle_knn_search(q, X, ld, dim, metric, base_adj, (uint32_t)N, stride, best.id, L,
                              out_ids, out_dist, &ndc, &nexp);
    return n;
}

/* ------------------------------------------------------------------ */
/* MIPS -> L2 (the standard transformation Section 4.3.1 points to).    */
/* ------------------------------------------------------------------ */

/*
 * Appends one coordinate to every base vector so that squared L2 ranks
 * like inner product: with n(x) = |x|^2 and M = max_x n(x),
 * x' = (x, sqrt(M - n(x))) has |x'|^2 = M for every row, and a query
 * q' = (q, 0) gives |q' - x'|^2 = |q|^2 + M - 2 <q, x>, which for a fixed q
 * orders the rows as -<q, x> does.  n(x) is the canonical FP32 squared
 * length (oracle_distance of x to the zero vector), sqrtf is correctly
 * rounded.  Output rows have ld_out >= dim + 4 floats: x, the extra
 * coordinate, then zeros up to dim + 4.  *max_norm2 receives M.
 */
int oracle_mips_to_l2(const float* X, uint64_t n, uint64_t ld, uint32_t dim, float* out,
                      uint64_t ld_out, float* max_norm2)
{
    if (!X || !out || dim == 0 || ld_out < (uint64_t)dim + 4 || n == 0) return -1;
    float* zero = (float*)calloc(dim, sizeof(float));
    float* nrm = (float*)malloc(sizeof(float) * n);
    if (!zero || !nrm) { free(zero); free(nrm); return -1; }
    float M = 0.0f;
    for (uint64_t i = 0; i < n; ++i) {
        nrm[i] = oracle_distance(X + i * ld, zero, dim, ORC_L2);
        if (nrm[i] > M) M = nrm[i];
    }
    for (uint64_t i = 0; i < n; ++i) {
        float* o = out + i * ld_out;
        for (uint32_t t = 0; t < dim; ++t) o[t] = X[i * ld + t];
        o[dim] = sqrtf(M - nrm[i]);
        for (uint64_t t = (uint64_t)dim + 1; t < ld_out; ++t) o[t] = 0.0f;
    }
    if (max_norm2) *max_norm2 = M;
    free(zero);
    free(nrm);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Ground truth: exact k-NN in FP64 by brute force.                     */
/* ------------------------------------------------------------------ */

typedef struct {
    double d;
    uint32_t id;
} ent64_t;

static int ent64_cmp(const void* pa, const void* pb)
{
    const ent64_t* x = (const ent64_t*)pa;
    const ent64_t* y = (const ent64_t*)pb;
    if (x->d < y->d) return -1;
    if (x->d > y->d) return 1;
    return x->id < y->id ? -1 : (x->id > y->id ? 1 : 0);
}

typedef struct {
    const float* X;
    uint64_t n, ld;
    uint32_t dim;
    int metric;
    const float* Q;
    uint64_t ldq;
    uint32_t k;
    const uint64_t* exclude;
    uint32_t* out_ids;
    double* out_dist;
} bf_ctx;

static double dist64(const float* a, const float* b, uint32_t dim, int metric)
{
    double s = 0.0;
    for (uint32_t t = 0; t < dim; ++t) {
        if (metric == ORC_L2) {
            double e = (double)a[t] - (double)b[t];
            s += e * e;
        } else {
            s += (double)a[t] * (double)b[t];
        }
    }
    if (metric == ORC_L2) return s;
    if (metric == ORC_IP) return -s;
    return 1.0 - s;
}

static void bf_range(void* p, uint64_t b, uint64_t e, int tid)
{
    (void)tid;
    bf_ctx* c = (bf_ctx*)p;
    ent64_t* buf = (ent64_t*)malloc(sizeof(ent64_t) * (c->n + 1));
    if (!buf) return;
    for (uint64_t qi = b; qi < e; ++qi) {
        const float* q = c->Q + qi * c->ldq;
        uint64_t ex = c->exclude ? c->exclude[qi] : UINT64_MAX;
        uint64_t m = 0;
        for (uint64_t v = 0; v < c->n; ++v) {
            if (v == ex) continue;
            buf[m++] = (ent64_t){dist64(q, c->X + v * c->ld, c->dim, c->metric), (uint32_t)v};
        }
        qsort(buf, m, sizeof(ent64_t), ent64_cmp);
        for (uint32_t t = 0; t < c->k; ++t) {
            c->out_ids[qi * c->k + t] = t < m ? buf[t].id : ORC_NONE;
            c->out_dist[qi * c->k + t] = t < m ? buf[t].d : INFINITY;
        }
    }
    free(buf);
}

/* Exact k nearest base rows of each query in FP64, (delta, id) order;
 * exclude[q] (nullable; UINT64_MAX = none) removes one base id per query. */
int oracle_bruteforce(const float* X, uint64_t n, uint64_t ld, uint32_t dim, int metric,
                      const float* Q, uint64_t nq, uint64_t ldq, uint32_t k,
                      const uint64_t* exclude, uint32_t* out_ids, double* out_dist,
                      int threads)
{
    bf_ctx c = {X, n, ld, dim, metric, Q, ldq, k, exclude, out_ids, out_dist};
    parallel_for(nq, threads, bf_range, &c);
    return 0;
}

/* FP64 distance, exposed for recall checks. */
double oracle_distance64(const float* a, const float* b, uint32_t dim, int metric)
{
    return dist64(a, b, dim, metric);
}

/* ------------------------------------------------------------------ */
/* Low-precision encodings for the precision form.                     */
/* ------------------------------------------------------------------ */

static uint32_t f2u(float f)
{
    uint32_t u;
    memcpy(&u, &f, 4);
    return u;
}

static float u2f(uint32_t u)
{
    float f;
    memcpy(&f, &u, 4);
    return f;
}

/* FP32 -> bfloat16, round to nearest even; NaN stays a quiet NaN. */
uint16_t oracle_bf16_from_f32(float x)
{
    uint32_t u = f2u(x);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu))
        return (uint16_t)((u >> 16) | 0x0040u);
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7FFFu + lsb;
    return (uint16_t)(u >> 16);
}

float oracle_bf16_to_f32(uint16_t b)
{
    return u2f((uint32_t)b << 16);
}

/*
 * FP32 -> FP8 E4M3 (OCP "fn" layout: 1 sign, 4 exponent bits with bias 7,
 * 3 mantissa bits, no infinities, S.1111.111 = NaN, largest finite 448),
 * round to nearest even with saturation to +-448.  Values are decoded from
 * the definition: exponent field e > 0 gives (1 + m/8) * 2^(e-7), e = 0
 * gives (m/8) * 2^-6.  The encoder picks the representable value nearest
 * to x by exhaustive comparison (ties to the even code).
 */
float oracle_fp8_to_f32(uint8_t c)
{
    uint32_t s = c >> 7, e = (c >> 3) & 15u, m = c & 7u;
    if (e == 15 && m == 7) return NAN;
    float v = e ? ldexpf(1.0f + (float)m / 8.0f, (int)e - 7) : ldexpf((float)m / 8.0f, -6);
    return s ? -v : v;
}

uint8_t oracle_fp8_from_f32(float x)
{
    if (isnan(x)) return 0x7F;
    uint8_t sign = signbit(x) ? 0x80 : 0x00;
    double a = fabs((double)x);
    if (a >= 448.0) return sign | 0x7E;
    uint8_t best = 0;
    double bd = INFINITY;
    for (uint32_t c = 0; c <= 0x7E; ++c) {
        double v = (double)oracle_fp8_to_f32((uint8_t)c);
        double dd = fabs(v - a);
        if (dd < bd || (dd == bd && (c & 1u) == 0 && (best & 1u) == 1)) {
            bd = dd;
            best = (uint8_t)c;
        }
    }
    return sign | best;
}

/*
 * Per-vector FP8 quantisation: scale s = max|x| / 448 (1 for an all-zero
 * row), code_t = fp8(x_t * (448 / max|x|)), so x_t ~ s * decode(code_t).
 * Also writes the dequantised rows s * decode(code) in FP32 (nullable).
 */
int oracle_quantize_fp8(const float* X, uint64_t n, uint64_t ld, uint32_t dim,
                        uint8_t* codes, float* scales, float* deq)
{
    for (uint64_t i = 0; i < n; ++i) {
        const float* x = X + i * ld;
        float amax = 0.0f;
        for (uint32_t t = 0; t < dim; ++t) {
            float a = fabsf(x[t]);
            if (a > amax) amax = a;
        }
        float inv = amax > 0.0f ? 448.0f / amax : 1.0f;
        float s = amax > 0.0f ? amax / 448.0f : 1.0f;
        scales[i] = s;
        for (uint32_t t = 0; t < dim; ++t) {
            uint8_t c = oracle_fp8_from_f32(x[t] * inv);
            codes[i * dim + t] = c;
            if (deq) deq[i * ld + t] = s * oracle_fp8_to_f32(c);
        }
    }
    return 0;
}

/* BF16 rows and their FP32 values (nullable deq). */
int oracle_quantize_bf16(const float* X, uint64_t n, uint64_t ld, uint32_t dim,
                         uint16_t* codes, float* deq)
{
    for (uint64_t i = 0; i < n; ++i)
        for (uint32_t t = 0; t < dim; ++t) {
            uint16_t b = oracle_bf16_from_f32(X[i * ld + t]);
            codes[i * dim + t] = b;
            if (deq) deq[i * ld + t] = oracle_bf16_to_f32(b);
        }
    return 0;
}
