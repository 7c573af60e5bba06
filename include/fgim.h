/*
 * fgim.h -- C ABI of the MI355X (gfx950) FGIM merge library (libfgim.so).
 *
 * FGIM (Wu et al., "FGIM: a Fast Graph-based Indexes Merging Framework for
 * Approximate Nearest Neighbor Search", PACMMOD 2026) merges h proximity
 * graphs G_i = (V_i, E_i), built over disjoint vector sets X_i with one
 * distance delta, into one graph over X = U X_i (problem definition
 * "Merging Graph-based Indexes for ANNS", Section 2.1).  It runs in three
 * stages (Section 3.3): PGs -> k-NNG by cross-querying (Section 4.1,
 * Algorithm 2), k-NNG refinement with indegree repair (Section 4.2,
 * Algorithms 3 and 4) and k-NNG -> PG by neighbour selection plus reverse
 * edges (Section 4.3, Algorithm 5).
 *
 * Conventions shared by every entry point:
 *  - Ids are uint32.  Global id of local vertex v of sub-index i is
 *    phi_i(v) = subs[i].row_offset + v (Section 4.1.3).  FGIM_NONE pads a
 *    short list; its distance slot holds +inf.
 *  - delta is squared L2, -<a,b> (inner product) or 1 - <a,b> (cosine; the
 *    caller passes unit vectors, the library never normalises).  Distances
 *    are FP32, summed in one fixed order: coordinates in chunks of 4 added
 *    left to right with fused multiply-adds, chunk sums combined by a stride
 *    tree over the chunk count padded to a power of two, -0 turned into +0.
 *  - Every list is sorted by (delta ascending, id ascending); ties are
 *    broken by id everywhere.
 *  - Pointers marked "device" are HIP device pointers; the caller owns all
 *    buffers and the library never frees them.  Temporary buffers come from
 *    a per-device scratch arena that the library keeps between calls (see
 *    fgim_release_scratch).
 *  - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream).
 *    Argument errors are returned before anything is enqueued.  Calls that
 *    must report FGIM_ERR_GRAPH (or fill a host-side result) synchronise the
 *    stream before returning; the others return with the work in flight.
 *  - With precision FGIM_FP32 the outputs do not depend on launch
 *    configuration (lanes per distance, waves per CU, visited-cache size):
 *    they are bit-identical across runs and tuning choices.
 *  - Outputs are undefined after any error.  Calls on one device share its
 *    scratch arena: they run one at a time on the host (other threads wait),
 *    and each call's device work starts after that of the previous call.
 *    The only other state kept between calls is the tuner's cache (used
 *    with autotune = 1 only) and the refinement's buffer demand seen so far
 *    (it sizes buffers and never changes a result).
 */
#ifndef FGIM_H
#define FGIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FGIM_NONE 0xFFFFFFFFu
#define FGIM_MAX_DIM 4096u
#define FGIM_MAX_K 128u       /* k, R */
#define FGIM_MAX_L 256u       /* beam width */
#define FGIM_MAX_STRIDE 128u  /* adjacency row stride */
#define FGIM_MAX_STREAM_BATCHES 4096u /* vertex ranges of a streamlined round */

typedef enum {
    FGIM_OK = 0,
    FGIM_ERR_INVALID_ARG = 1,   /* null pointer, size out of range, bad ranges */
    FGIM_ERR_GRAPH = 2,         /* adjacency id out of range, self-loop or duplicate */
    FGIM_ERR_OUT_OF_MEMORY = 3, /* scratch allocation failed */
    FGIM_ERR_DEVICE = 4,        /* a HIP call failed */
    FGIM_ERR_UNSUPPORTED = 5    /* valid request this build does not handle */
} fgim_status;

typedef enum { FGIM_L2 = 0, FGIM_IP = 1, FGIM_COSINE = 2 } fgim_metric;

/* Arithmetic of the candidate scoring.  FP32 is the exact (parity) form.
 * BF16 and FP8_E4M3 score candidates on a low-precision copy of the base
 * vectors (round-to-nearest-even BF16; OCP E4M3 with one FP32 scale per
 * vector, scale = max|x| / 448) and re-score each node's best candidates
 * on the FP32 rows before any list is written. */
typedef enum { FGIM_FP32 = 0, FGIM_BF16 = 1, FGIM_FP8_E4M3 = 2 } fgim_precision;

/* One input proximity graph G_i (problem definition, Section 2.1). */
typedef struct {
    uint64_t row_offset;   /* phi_i offset: global id / base row of local vertex 0 */
    uint32_t n;            /* |V_i|, >= 1 */
    uint32_t adj_stride;   /* row stride of adj (the input degree bound R_in), 1..128 */
    const uint32_t* adj;   /* device, n x adj_stride local ids, FGIM_NONE padded */
    uint32_t entry;        /* local id of the entry point ep_i (< n) */
} fgim_subindex;

/* The base vectors X and the h input graphs.  Sub-indexes must be given in
 * ascending row_offset order and tile [0, n_total) without gaps. */
typedef struct {
    const float* base;          /* device, n_total rows of ld floats; 16-byte aligned */
    uint64_t n_total;           /* sum of n_i, < 0xFFF00000 */
    uint32_t dim;               /* d: multiple of 4, 4..FGIM_MAX_DIM */
    uint64_t ld;                /* row stride in floats: multiple of 4, >= dim */
    fgim_metric metric;
    const fgim_subindex* subs;  /* host array of h entries */
    uint32_t h;                 /* number of sub-indexes, >= 1 */
    /* Optional low-precision copy for the BF16 / FP8 forms (device,
     * dense n_total x dim, as written by fgim_quantize).  When NULL the
     * library quantises into scratch inside the call. */
    const void* base_lp;
    const float* base_lp_scale; /* device, n_total FP8 scales (FP8 only) */
    /* Validity of the ID mapping phi (Section 4.1.3; deletions and
     * overlapping copies, Exp. 8): device, n_total bytes, 1 = retained,
     * 0 = deleted or a duplicate to drop; NULL = every vertex retained.
     * A dropped vertex gets an empty row (FGIM_NONE, +inf, degree 0) and is
     * never a neighbour in any output; the cross-query searches still route
     * through it, since it is part of its input graph. */
    const uint8_t* valid;
} fgim_dataset;

typedef struct {
    uint32_t k;          /* k-NNG degree, 1..FGIM_MAX_K (Algorithm 2 "outdegree bound k") */
    uint32_t L;          /* cross-query beam width (Algorithm 1 pool size), 1..FGIM_MAX_L */
    uint32_t R;          /* output PG degree, 1..FGIM_MAX_K (Algorithm 5 bound) */
    uint32_t rounds;     /* refinement iterations I_max (Algorithm 3) */
    fgim_precision precision;
    uint32_t rerank;     /* candidates per search re-scored in FP32; 0 -> min(L, 2k) */
    uint32_t k_rev;      /* cap of each reverse list in refinement; 0 -> k */
    int autotune;        /* 0: L as given; 1: the tuner may lower L to the
                            minimum-querying bound of Section 4.1.2 and picks
                            the launch shape */
    /* Launch shape (0 = choose automatically).  None of these changes an
     * FP32 result bit.  The automatic shape gives each lane four chunks of
     * four coordinates (fewer below d = 64; at most 64 lanes, so more above
     * d = 1024), 32 waves per CU and 1024 visited
     * slots for L <= 32, else 2048; when the graphs searched have a mean
     * out-degree of at most 12 (each graph weighted by the searches run in
     * it), two chunks per lane and 1024 slots. */
    uint32_t lanes_per_dist;   /* lanes that share one distance: 1..64, power of 2 */
    uint32_t waves_per_cu;     /* resident waves per compute unit of the beam kernel */
    uint32_t visited_slots;    /* entries of the per-wave LDS visited cache (power of 2) */
    uint32_t flags;            /* FGIM_FLAG_* */
    /* Neighbour-selection rule of stage 3 (Section 4.3.1 names RNG and, as
     * swap-ins, alpha-RNG and tau-MNG); FGIM_SELECT_RNG is Algorithm 5. */
    uint32_t select_rule;      /* FGIM_SELECT_* */
    float select_param;        /* alpha (>= 1) or tau (>= 0); unused by RNG */
    /* Refinement schedule (Section 4.2.1).  0 or 1: synchronous rounds,
     * every vertex visited against one snapshot.  B in 2..FGIM_MAX_STREAM_
     * BATCHES: streamlined rounds, which visit the vertex ranges
     * [t n / B, (t + 1) n / B), t = 0 .. B-1, in turn; each range's Visit and
     * Update read the lists as the earlier ranges left them.  Deterministic
     * for every B. */
    uint32_t stream_batches;
    /* Synchronous rounds with the MFMA join: the Update runs in this many
     * vertex chunks (at most FGIM_MAX_STREAM_BATCHES) that share one buffer
     * of screened pairs; every chunk joins against the same snapshot, so the
     * count changes no result, only the buffer size.  0: as many as keep
     * the buffer within 2^28 pairs (2 GiB). */
    uint32_t update_chunks;
} fgim_params;

/* Selection rules: whether a kept neighbour w, at delta(w, v) from the
 * candidate v, leaves v selectable for u (delta(u, v) from u).  A v with
 * indegree T(v) = 1 is kept under every rule.
 *  RNG:   delta(u,v) < delta(w,v).
 *  ALPHA: |u-v| < alpha |w-v| on Euclidean distances (Vamana's robust
 *         prune); on delta (squared L2, or half of it for cosine on unit
 *         vectors) delta(u,v) < fl(fl(alpha * alpha) * delta(w,v)).
 *  TAU:   w occludes v when |w-v| < |u-v| - 3 tau (the tau-monotonic
 *         graph's rule); v survives when e(u,v) < fl(e(w,v) + fl(3 tau)),
 *         e = sqrt(delta) (L2) or sqrt(2 delta) (cosine), correctly rounded.
 * ALPHA and TAU need a metric distance: L2 or cosine (for inner product,
 * transform the data with fgim_mips_to_l2 and merge under L2). */
#define FGIM_SELECT_RNG 0u
#define FGIM_SELECT_ALPHA 1u
#define FGIM_SELECT_TAU 2u

#define FGIM_FLAG_NO_REPAIR 1u     /* refinement without indegree repair (test hook) */
#define FGIM_FLAG_NO_GRAPH_CAPTURE 2u /* run refinement rounds eagerly, not as a hipGraph */
#define FGIM_FLAG_NO_MFMA_SCREEN 4u /* score every join pair and every occlusion pair of the
                                       neighbour selection in FP32 instead of screening the
                                       tiles on MFMA first (same result; test hook) */
#define FGIM_FLAG_MIN_BUFFERS 8u   /* start the refinement's screened-pair and proposal buffers
                                      at their minimum (2^16 entries), ignoring the demand seen
                                      before, so that the overflow-and-rerun path runs (test hook) */

/* Per-call counters; passing a non-NULL stats pointer synchronises the
 * stream at the end of the call. */
typedef struct {
    double ms_stage[3];       /* wall time of stage 1, 2, 3 on the stream (hipEvents) */
    double ms_beam_kernel;    /* duration of the stage-1 beam-search kernel alone */
    uint64_t ndc;             /* distance computations of the beam searches */
    uint64_t expansions;      /* pool entries expanded by the beam searches */
    uint64_t searches;        /* beam searches run */
    uint64_t proposals;       /* join proposals that passed the worst-entry screen */
    uint64_t repaired;        /* zero-indegree vertices given an in-edge */
    uint64_t rechecked;       /* join pairs re-scored in FP32 after the MFMA screen */
    uint32_t L_used;          /* beam width actually used */
    uint32_t lanes_per_dist;  /* launch shape actually used */
    uint32_t waves_per_cu;
    uint32_t visited_slots;
    double ms_tune;           /* time spent on tuner trial launches (autotune=1; 0 on a cache hit) */
    uint64_t repair_batches;  /* speculative batches of the indegree-repair passes */
    uint64_t repair_alone;    /* repair steps that needed more than one attempt (run alone) */
    uint32_t refine_attempts; /* refinement runs: above 1 when a pair or proposal buffer
                                 overflowed and the rounds ran again with larger ones */
} fgim_stats;

/*
 * Stage 1, PGs -> k-NNG (Section 4.1, Algorithm 2).  For every vertex u of
 * every G_i: the local candidates C+(u) are u's out-neighbours in G_i
 * (Section 4.1.1, "Local Candidate Neighbors"); every other G_j is searched
 * with Algorithm 1 (beam width L, from ep_j: "cross-querying", "Cross
 * Candidate Neighbors"); the union is mapped to global ids by phi, sorted,
 * and its first k entries form row phi_i(u) of the k-NNG.
 * Outputs (device, n_total x k): knn_ids, knn_dist (canonical FP32 delta).
 * Errors: FGIM_ERR_INVALID_ARG (arguments), FGIM_ERR_GRAPH (bad adjacency,
 * checked on the device; the call then synchronises).
 */
fgim_status fgim_cross_query(const fgim_dataset* data, const fgim_params* params,
                             uint32_t* knn_ids, float* knn_dist, fgim_stats* stats,
                             void* stream);

/*
 * Stage 1 as fgim_cross_query, for callers that cannot allocate device
 * memory (code under stream capture, serving loops, harnesses that forbid
 * hipMalloc): it allocates nothing.  Its temporary state -- the work-queue
 * head, the error flag, the counters and the sub-index table, 131,328 bytes
 * in all -- lives in a fixed array in the library's device memory, one per
 * GPU, held until the process ends.  Calls on one GPU share that array and
 * run one at a time (a per-device host lock); each clears what it needs
 * before its launch, and the array keeps the last call's contents.
 * Limits: autotune must be 0 (the tuner's trial launches need memory), the
 * BF16 / FP8 forms need data->base_lp (and base_lp_scale for FP8), and
 * h <= 4096.  Outputs are bit-identical to fgim_cross_query's with the same
 * arguments.  Synchronises the stream before returning.
 * Errors: FGIM_ERR_INVALID_ARG (arguments, or a limit above), FGIM_ERR_GRAPH
 * (bad adjacency), FGIM_ERR_DEVICE (the array's address lookup failed).
 */
fgim_status fgim_cross_query_noalloc(const fgim_dataset* data, const fgim_params* params,
                                     uint32_t* knn_ids, float* knn_dist, void* stream);

/*
 * Stage 2, k-NNG refinement (Section 4.2, Algorithms 3 and 4), run as
 * `rounds` rounds.  Each round: Visit splits each list and its reverse
 * lists into new and old candidates, Update proposes every cross-sub-index
 * pair of C_n^2 U C_n x C_o to both ends, every list keeps its k best of its
 * entries and the proposals, then indegree repair links each zero-indegree
 * vertex into a neighbour's list.  A synchronous round does this for all
 * vertices at once; a streamlined one (params->stream_batches > 1) for one
 * vertex range after another, each on the lists the earlier ranges left
 * (Section 4.2.1).  All input entries count as new.  knn_ids / knn_dist (device, n_total x k) are read and rewritten;
 * indegree (device, n_total, nullable) receives T after the last round.
 * Errors: FGIM_ERR_INVALID_ARG (arguments), FGIM_ERR_GRAPH (a list id that
 * is neither FGIM_NONE nor below n_total; checked on the device before any
 * list is changed, the call then synchronises).
 */
fgim_status fgim_refine(const fgim_dataset* data, const fgim_params* params,
                        uint32_t* knn_ids, float* knn_dist, uint32_t* indegree,
                        fgim_stats* stats, void* stream);

/*
 * Indegree repair alone (Section 4.2.2, Algorithm 4) on a k-NNG whose rows
 * are sorted by (distance, id) with FGIM_NONE padding at the end: T is the
 * indegree histogram of the lists; every v* with T(v*) = 0, in ascending id,
 * tries its neighbours v from the closest and enters N(v) in place of the
 * farthest entry that is not already a repair edge and whose indegree
 * exceeds 1 (or takes a free slot), flagged as a repair edge.  The same pass
 * ends every refinement round of fgim_refine.
 * In/out (device, n x k): knn_ids, knn_dist.  indegree (device, n,
 * nullable) receives T after the pass; *repaired (host, nullable) the number
 * of vertices that gained an in-edge (the call then synchronises).
 * Errors: FGIM_ERR_INVALID_ARG (arguments), FGIM_ERR_GRAPH (an id >= n,
 * checked before any list changes; the call synchronises for it).
 */
fgim_status fgim_repair(uint32_t* knn_ids, float* knn_dist, uint64_t n, uint32_t k,
                        uint32_t* indegree, uint64_t* repaired, void* stream);

/*
 * Stage 3, k-NNG -> PG (Section 4.3, Algorithm 5).  Neighbour selection
 * keeps v in N(u) (closest first) when T(v) = 1 or delta(u,v) < delta(w,v)
 * for every kept w, up to R; connectivity enhancement then adds the reverse
 * of every selected edge, sorts and keeps the first R.
 * Inputs (device): knn_ids / knn_dist (n_total x k), indegree T (n_total).
 * Outputs (device): pg_ids (n_total x R, FGIM_NONE padded), pg_deg (n_total).
 */
fgim_status fgim_prune(const fgim_dataset* data, const fgim_params* params,
                       const uint32_t* knn_ids, const float* knn_dist,
                       const uint32_t* indegree, uint32_t* pg_ids, uint32_t* pg_deg,
                       void* stream);

/*
 * The three stages in one call (Section 3.3).  Outputs: pg_ids, pg_deg as
 * fgim_prune; *entry (host) = global id of the merged graph's entry point,
 * the entry of the largest sub-index (lowest index on ties).  With validity
 * flags, when that entry is dropped: the smallest retained id of the same
 * sub-index; a sub-index with no retained vertex is passed over for the next
 * largest; FGIM_NONE when nothing is retained.  Synchronises.
 */
fgim_status fgim_merge(const fgim_dataset* data, const fgim_params* params,
                       uint32_t* pg_ids, uint32_t* pg_deg, uint32_t* entry,
                       fgim_stats* stats, void* stream);

/*
 * Algorithm 1 (KNNSearch) for a batch of queries on one graph, used to
 * evaluate a merged index (Recall@k, Section 2.1).  Graph: adj (device,
 * n x stride ids into base), entry.  Queries (device, nq rows of ldq
 * floats).  Outputs (device, nq x topk): the first topk pool entries.
 * topk <= L.
 */
fgim_status fgim_search(const float* base, uint64_t n, uint32_t dim, uint64_t ld,
                        fgim_metric metric, const uint32_t* adj, uint32_t stride,
                        uint32_t entry, const float* queries, uint64_t nq, uint64_t ldq,
                        uint32_t L, uint32_t topk, uint32_t* out_ids, float* out_dist,
                        void* stream);

/*
 * Measurement aid, not a step of the method: reads `bytes` bytes of `data`
 * (device, 16-byte aligned, bytes a multiple of 16; may be NULL when bytes
 * is 0) once with wide
 * coalesced loads spread over every compute unit, and writes the XOR of all
 * its 32-bit words to *checksum (device; zeroed first).  Its duration is the
 * read-stream bandwidth that bounds a kernel which only reads, such as the
 * stage-1 beam search.  Asynchronous on `stream`.
 * Errors: FGIM_ERR_INVALID_ARG.
 */
fgim_status fgim_read_stream(const void* data, uint64_t bytes, uint32_t* checksum, void* stream);

/*
 * Low-precision copy for the BF16 / FP8 forms.  BF16: codes = uint16
 * [n x dim]; FP8_E4M3: codes = uint8 [n x dim] and scales (device, n).
 * Same encodings as described at fgim_precision.
 */
fgim_status fgim_quantize(const float* base, uint64_t n, uint32_t dim, uint64_t ld,
                          fgim_precision precision, void* codes, float* scales,
                          void* stream);

/*
 * HNSW-adaptive merging (Section 4.3.3): the upper layers of an HNSW index
 * over the merged base graph (layer 0).  levels (device, n bytes) holds each
 * vertex's level, drawn by the caller from HNSW's level distribution
 * (floor(-ln U / ln M) is the usual draw); layer l = 1..max_level holds the
 * vertices with level >= l, layer_count[l - 1] of them (host array: the
 * caller counts them to size its buffers; a mismatch is an error).  Each
 * layer is built in one batch: the ef nearest other members of every
 * member (exact, canonical FP32), HNSW's neighbour heuristic up to M (the
 * RNG rule of Algorithm 5 without the indegree exemption), the first 2M of
 * those neighbours and the reverse edges by (delta, id), and the heuristic
 * again up to M.  Outputs (device), layers concatenated in order:
 * layer_ids (members, ascending), layer_adj (M global ids per member,
 * FGIM_NONE padded); *top (host) = the smallest id of the highest layer,
 * the search's entry point (FGIM_NONE when max_level = 0).  M in 1..64,
 * ef in M..128.  Synchronises.
 * Errors: FGIM_ERR_INVALID_ARG (arguments, a level above max_level, wrong
 * layer_count).
 */
fgim_status fgim_hnsw_layers(const float* base, uint64_t n, uint32_t dim, uint64_t ld, fgim_metric metric,
                             const uint8_t* levels, uint32_t max_level, uint32_t M, uint32_t ef,
                             const uint64_t* layer_count, uint32_t* layer_ids, uint32_t* layer_adj,
                             uint32_t* top, void* stream);

/*
 * Search of the hierarchy that fgim_hnsw_layers builds: greedy descent from
 * top through layers max_level..1 (each step moves to the neighbour closest
 * to the query by (delta, id) while it beats the current vertex), then
 * Algorithm 1 with beam width L on the base graph (base_adj, n x stride)
 * from the vertex reached.  Outputs (device, nq x topk) as fgim_search.
 * Errors: FGIM_ERR_INVALID_ARG, FGIM_ERR_GRAPH (an id out of range in the
 * base graph or the layers; checked before the search, which then
 * synchronises).
 */
fgim_status fgim_search_layers(const float* base, uint64_t n, uint32_t dim, uint64_t ld, fgim_metric metric,
                               const uint32_t* base_adj, uint32_t stride, const uint32_t* layer_ids,
                               const uint32_t* layer_adj, const uint64_t* layer_count, uint32_t max_level,
                               uint32_t M, uint32_t top, const float* queries, uint64_t nq, uint64_t ldq,
                               uint32_t L, uint32_t topk, uint32_t* out_ids, float* out_dist, void* stream);

/*
 * The standard transformation of maximum-inner-product search to L2 that
 * Section 4.3.1 points to, so that the distance-based selection rules apply
 * to inner-product data: with n(x) = |x|^2 (canonical FP32 sum) and
 * M = max n(x), row x becomes x' = (x, sqrt(M - n(x)), 0, 0, 0): every x'
 * has squared length M, and a query padded as q' = (q, 0, 0, 0, 0) gives
 * |q' - x'|^2 = |q|^2 + M - 2 <q, x>, which orders rows as -<q, x> does.
 * Merge the transformed rows under FGIM_L2.
 * Input base (device, n rows of ld floats, dim a multiple of 4); output out
 * (device, n rows of ld_out >= dim + 4 floats, 16-byte aligned; only the
 * first dim + 4 floats of a row are written); *max_norm2 (device, 1 float)
 * receives M.  The square root is correctly rounded.
 * Errors: FGIM_ERR_INVALID_ARG.
 */
fgim_status fgim_mips_to_l2(const float* base, uint64_t n, uint32_t dim, uint64_t ld, float* out,
                            uint64_t ld_out, float* max_norm2, void* stream);

/* ceil((k - min_local) / (h - 1)), at least 1: the smallest L for which
 * every vertex still collects k candidates (minimum querying strategy,
 * Section 4.1.2).  0 when h < 2. */
uint32_t fgim_min_beam_width(uint32_t k, uint32_t min_local, uint32_t h);

/*
 * Scratch memory.  Every call takes its temporary buffers from a device
 * arena that the library keeps between calls (it grows to the largest total
 * a call has needed; until then the excess comes from the device's
 * stream-ordered memory pool).  Calls on one device therefore run one at a
 * time on the host, and a call's device work starts after that of the
 * previous call.  fgim_release_scratch waits for the current device's last
 * call to finish on the device and frees its arena; the next call starts a
 * new one.  Errors: FGIM_ERR_DEVICE (no device, or a HIP failure).
 */
fgim_status fgim_release_scratch(void);

const char* fgim_status_string(fgim_status status);
/* Detail of the last error on the calling thread ("" if none). */
const char* fgim_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FGIM_H */
