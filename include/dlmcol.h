/*
 * dlmcol.h -- C ABI of the MI355X (gfx950) population graph-colouring hot
 * path of the deep-learning guided memetic colouring method (Goudet, Grelier
 * and Hao, "A deep learning guided memetic framework for graph coloring
 * problems").
 *
 * Conventions for every call:
 *   - Return value: DLM_OK (0) or a negative DLM_E_* status.  The message of
 *     the last failure on the calling thread is returned by dlm_last_error().
 *     On failure nothing has been launched after the failing check and the
 *     contents of output buffers are unspecified.
 *   - Pointers named *_dev are device (HBM) pointers owned by the caller; the
 *     library never frees or keeps them after the call returns.  Pointers
 *     named *_host are host pointers read synchronously during the call.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *     device work is asynchronous on that stream: outputs are valid once the
 *     caller synchronises it.
 *   - Colourings are int16 [count][n] row-major; colours are 0..k-1.
 *   - Randomness is counter based (Philox4x32-10 keyed by the 64-bit seed), so
 *     an individual's result depends only on (inputs, seed, its global index),
 *     never on the population size, launch shape or table storage.
 */
#ifndef DLMCOL_H
#define DLMCOL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DLM_ABI_VERSION 2

#define DLM_OK 0
#define DLM_E_INVAL (-1)       /* bad argument (null pointer, size, range, CSR rule) */
#define DLM_E_NOMEM (-2)       /* device allocation failed */
#define DLM_E_HIP (-3)         /* a HIP runtime call or kernel launch failed */
#define DLM_E_UNSUPPORTED (-4) /* valid request beyond what this library supports */

#define DLM_NSTATS 8 /* per-individual counters written by the tabu calls */

/* Version of this ABI (DLM_ABI_VERSION of the build). */
int dlm_abi_version(void);

/* Message of the last failure on the calling thread ("" if none). */
const char* dlm_last_error(void);

/* ------------------------------------------------------------------------
 * Graph ingest.  The graph G = (V, E) of the colouring problems (Section 1 of
 * the paper), shared read-only by every search in device memory (Section 2.2:
 * the graph lives in global memory, shared by all tabu runs).
 * ---------------------------------------------------------------------- */
typedef struct dlm_graph dlm_graph; /* opaque, immutable after creation */

#define DLM_G_BITSET 0x1u /* also keep bitset adjacency rows: not built (DLM_E_UNSUPPORTED) */

/*
 * Validate and upload an undirected simple graph in CSR form.
 *   n            number of vertices, 1 <= n <= 32767
 *   row_ptr_host int32[n+1], row_ptr[0] = 0, non-decreasing
 *   col_idx_host int32[row_ptr[n]]: both directions of every edge, each row
 *                strictly ascending, indices in [0, n), no self loops,
 *                symmetric
 *   weights_host int32[n] vertex weights w_v > 0 (weighted problem), or NULL;
 *                a weighted graph also stores the greedy start order of
 *                Section 2.1 (weight descending, degree descending, index
 *                ascending), computed here once
 *   flags        0, or DLM_G_BITSET (returns DLM_E_UNSUPPORTED: this library
 *                streams CSR rows only); other bits are DLM_E_INVAL
 *   stream       the uploads are ordered on it; the call synchronises it
 *                before returning, so the host arrays may be freed at once
 * On success *out owns device copies (allocated on the current device, which
 * every later call on the graph must use); release with dlm_graph_destroy.
 * Errors: DLM_E_INVAL for any CSR rule broken, DLM_E_UNSUPPORTED,
 * DLM_E_NOMEM, DLM_E_HIP.
 */
int dlm_graph_create(int32_t n, const int32_t* row_ptr_host, const int32_t* col_idx_host,
                     const int32_t* weights_host, uint32_t flags, void* stream, dlm_graph** out);
int dlm_graph_destroy(dlm_graph* g);
/* n, number of CSR entries (2|E|) and the maximum degree; any output may be NULL. */
int dlm_graph_info(const dlm_graph* g, int32_t* n, int64_t* nnz, int32_t* max_deg);

/* ------------------------------------------------------------------------
 * Population initialisation.
 *   DLM_INIT_RANDOM (k-COL, Section 2.7): colour of vertex v of individual i =
 *     floor(w0 * k / 2^32), w0 = Philox(seed; ind_base+i, 0, v, 0x80000002).
 *   DLM_INIT_GREEDY (WVCP, Section 2.1): vertices by weight descending, then
 *     degree descending, then index; each takes a random already-used colour
 *     that creates no conflict (uniform pick among them, Philox counter
 *     (ind, 0, v, 0x80000008)), else opens a new colour numbered by creation
 *     order.  k is not used in this mode; k_used_dev receives the number of
 *     colours each individual used, and a search that follows needs k at
 *     least their maximum.  Needs a weighted graph.
 *   colors_dev  int16[pop][n] output
 *   k_used_dev  int32[pop] output: colours used (greedy) or k (random); may
 *               be NULL
 * ---------------------------------------------------------------------- */
#define DLM_INIT_RANDOM 0
#define DLM_INIT_GREEDY 1
int dlm_init_population(const dlm_graph* g, int32_t k, int32_t pop, uint64_t seed,
                        int32_t ind_base, int32_t mode, int16_t* colors_dev,
                        int32_t* k_used_dev, void* stream);

/* ------------------------------------------------------------------------
 * Population TabuCol (k-COL local search, Section 2.7; TabuCol with the
 * gamma table of its efficient implementation).  One workgroup per
 * individual; each keeps the n x k table gamma[v][c] = number of neighbours
 * of v coloured c, plus the tabu expiry of every (v, c).
 *
 * Iteration t (t = 0, 1, ...) while t < max_iters and f > 0:
 *   candidates: (v, c) with gamma[v][col v] > 0 (v in conflict), c != col v,
 *     delta = gamma[v][c] - gamma[v][col v];
 *   admissible: not tabu (expiry <= t) or f + delta < f_best (aspiration);
 *   choice: lexicographic minimum of (delta, h, v, c), h = word 0 of
 *     Philox(seed; ind, t, v, c); no admissible move => no-op iteration;
 *   move: col v = c, f += delta, (v, old colour) tabu until
 *     t + L + min(floor(ten_num * f / ten_den), 32757) with
 *     L = floor(w0 * ten_rand / 2^32), w0 = Philox(seed; ind, t, 0, 0x80000001);
 *   the best colouring met (smallest f) is kept.
 * ---------------------------------------------------------------------- */
#define DLM_TABLE_AUTO 0       /* WAVE8 when it holds the individual and block is 0 or 64; otherwise LDS16 or
                                  SPLIT8, whichever keeps more workgroups per CU; GLOBAL16 if neither fits */
#define DLM_TABLE_LDS16 1      /* 32-bit word per (v,c): gamma 16 bits | tabu 16 bits, LDS */
#define DLM_TABLE_LDS32 2      /* 64-bit word per (v,c): gamma int32 | tabu expiry, LDS */
#define DLM_TABLE_GLOBAL16 3   /* packed 16-bit words in device memory (large n*k) */
#define DLM_TABLE_SPLIT16 4    /* gamma 16 bits in LDS, tabu 16 bits in device memory */
#define DLM_TABLE_SPLIT8 5     /* gamma 8 bits in LDS, tabu 16 bits in device memory; an individual
                                  whose colour classes would pass 255 vertices is rerun from its
                                  start with GLOBAL16 (same results) */
#define DLM_TABLE_WAVE8 6      /* one wavefront (block 64) per individual, all in LDS: a byte per (v,c)
                                  holding gamma (7 bits) and a flag for "current colour or tabu", and a
                                  list of the live tabu pairs with their expiries; needs k <= 256 and
                                  n * kp <= 2^17.  An individual whose colour classes would pass 127
                                  vertices, or whose live tabu pairs would overflow the list, is rerun
                                  from its start with GLOBAL16 (same results) */

typedef struct dlm_tabu_params {
  int32_t k;          /* colours, 1 <= k <= 32767 */
  int32_t max_iters;  /* iteration budget T, 0 <= T <= 2^30 */
  int32_t ten_num;    /* tenure slope numerator (6 for 0.6 f) */
  int32_t ten_den;    /* tenure slope denominator (10), > 0 */
  int32_t ten_rand;   /* L uniform in [0, ten_rand), 1..1024 */
  int32_t ind_base;   /* global index of row 0 of the population */
  uint64_t seed;      /* Philox key */
  int32_t block;      /* threads per workgroup: 0 = auto (64 with the WAVE8 table; otherwise 256, or
                         512 when AUTO storage fits only one individual per CU), else 64, 128, 256,
                         512 or 1024 (WAVE8 takes only 0 or 64) */
  int32_t table;      /* DLM_TABLE_* storage of the n x k table */
  int32_t trace_cap;  /* records per individual in trace_dev (0 = none) */
  int32_t reserved;   /* must be 0 */
} dlm_tabu_params;

/*
 * Device workspace a dlm_tabu_batch call with these arguments needs, in
 * bytes (0 for the LDS tiers).  The automatic table and block are resolved
 * as the call resolves them, on the current device.  The device-memory tiers
 * need their tables (pop * (n + 1) * kp entries of 4 bytes for GLOBAL16, 2
 * for SPLIT16 and SPLIT8); SPLIT8 adds a copy of the start colourings and
 * the rerun tables (at most 2 per CU and 1 GiB).
 * Errors: as dlm_tabu_batch's argument checks.
 */
int dlm_tabu_workspace_bytes(const dlm_graph* g, const dlm_tabu_params* p, int32_t pop, size_t* bytes);

/*
 * Run TabuCol on every individual of a population.
 *   pop          number of individuals (0 is a no-op)
 *   colors_dev   int16[pop][n]: in = start colouring S^O, out = best S'
 *   f_best_dev   int32[pop]: conflicts of the returned colouring
 *   iters_dev    int32[pop]: iterations run (stops early at f = 0)
 *   stats_dev    int64[pop][DLM_NSTATS] or NULL: 0 moves, 1 no-ops, 2 sum over
 *                iterations of the number of conflicting vertices scanned,
 *                3 sum over moves of deg(v*), 4 iterations whose minimum
 *                delta was shared by >= 2 admissible moves, 5 tenure-cap hits
 *   hash_dev     uint64[pop] or NULL: FNV-1a (64-bit) over the move records
 *                (v | c << 16 | (uint32)f_after << 32); a no-op records
 *                v = c = 0xffff
 *   trace_dev    int32[pop][trace_cap][2] or NULL: {v | c << 16, f_after} of
 *                the first trace_cap iterations
 *   workspace_dev, workspace_bytes  caller-owned device scratch, 256-byte
 *                aligned, at least dlm_tabu_workspace_bytes(g, p, pop) bytes
 *                (may be NULL when that is 0); its contents on entry do not
 *                matter, and it must not be shared with a call that overlaps
 *                this one.  The call allocates no device memory.
 * A start colouring holding a colour outside [0, k) is left untouched and its
 * individual gets f_best = iters = -1 (its stats and hash are not written).
 * Errors: DLM_E_INVAL (arguments, workspace missing, too small or
 * misaligned), DLM_E_UNSUPPORTED (table does not fit the requested storage),
 * DLM_E_HIP.
 */
int dlm_tabu_batch(const dlm_graph* g, const dlm_tabu_params* p, int32_t pop,
                   int16_t* colors_dev, int32_t* f_best_dev, int32_t* iters_dev,
                   int64_t* stats_dev, uint64_t* hash_dev, int32_t* trace_dev,
                   void* workspace_dev, size_t workspace_bytes, void* stream);

/*
 * dlm_tabu_batch for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, hosts that forbid hipMalloc): the
 * same search with the same arguments and bit-identical outputs, but its
 * workspace is a fixed array of DLM_STATIC_SCRATCH_BYTES in the library's
 * device code (one per GPU, held from the library's load until the process
 * ends) instead of a caller-owned buffer.  The call allocates nothing: no
 * hipMalloc, hipFree or allocating library routine.  The array's device
 * address is looked up once per device, on the first call made with that
 * device current.
 *   Every call on one GPU shares that GPU's array: calls that overlap on one
 *   GPU (two streams, two host threads) race and give undefined results;
 *   calls ordered on one stream, or separated by synchronisation, are safe.
 *   Nothing in the array needs clearing between calls: each launch writes
 *   every byte of the workspace it reads first.
 * Errors: as dlm_tabu_batch; DLM_E_UNSUPPORTED when the workspace this call
 * would need (dlm_tabu_workspace_bytes) exceeds DLM_STATIC_SCRATCH_BYTES, in
 * which case nothing is launched.
 */
#define DLM_STATIC_SCRATCH_BYTES (64ull << 20)
int dlm_tabu_batch_static(const dlm_graph* g, const dlm_tabu_params* p, int32_t pop,
                          int16_t* colors_dev, int32_t* f_best_dev, int32_t* iters_dev,
                          int64_t* stats_dev, uint64_t* hash_dev, int32_t* trace_dev, void* stream);

/* ------------------------------------------------------------------------
 * Uneven batches: the populations of many graphs (any mix of n, k and
 * iteration budgets) searched by one persistent launch.  Each item is a
 * dlm_tabu_batch call in all but the launch: same search, same outputs,
 * bit-identical results.  Work items (graph, individual) are taken
 * longest-first from an atomic queue by a grid sized to the device's
 * resident capacity; graphs whose table fits the LDS budget use the LDS16
 * table, graphs whose byte gamma alone fits use the SPLIT8 table (expiries in
 * device memory; an individual whose colour classes would pass 255 vertices is
 * rerun in place with the device-memory table, same results), the others the
 * device-memory table.  A plan captures the queue
 * reset and the persistent kernel into a hipGraph once; each launch replays
 * it on the caller's stream and searches whatever the item buffers hold.
 * The plan keeps the item pointers: buffers and graphs must outlive it.
 * ---------------------------------------------------------------------- */
typedef struct dlm_multi_item {
  const dlm_graph* g;
  int32_t k, max_iters, pop, ind_base;     /* as in dlm_tabu_params */
  int32_t ten_num, ten_den, ten_rand, reserved;
  uint64_t seed;
  int16_t* colors_dev;   /* int16[pop][n], in: start, out: best */
  int32_t* f_best_dev;   /* int32[pop] */
  int32_t* iters_dev;    /* int32[pop] */
  int64_t* stats_dev;    /* int64[pop][DLM_NSTATS] or NULL */
  uint64_t* hash_dev;    /* uint64[pop] or NULL */
} dlm_multi_item;

typedef struct dlm_multi_config {
  int32_t block;       /* threads per workgroup: 0 = 256, else 64, 128, 256 or 512 */
  int32_t lds_budget;  /* LDS bytes a graph's table may use (0 = device maximum) */
} dlm_multi_config;

typedef struct dlm_multi_plan dlm_multi_plan;

int dlm_multi_plan_create(const dlm_multi_item* items, int32_t count, const dlm_multi_config* cfg,
                          void* stream, dlm_multi_plan** out);
int dlm_multi_plan_launch(dlm_multi_plan* plan, void* stream);
/* grid size, dynamic LDS bytes, graphs using device memory for (part of)
 * their table, items */
int dlm_multi_plan_info(const dlm_multi_plan* plan, int32_t* grid, int32_t* lds_bytes,
                        int32_t* n_global, int32_t* total_items);
int dlm_multi_plan_destroy(dlm_multi_plan* plan);

/*
 * Autotuner: times every (block in {64,128,256,512}) x (LDS budget in
 * {1/4, 1/2, 1} of the device maximum) on scratch copies of the items'
 * colourings with at most calib_iters iterations per individual, and
 * returns the configuration with the most iterations per second in *best.
 * rates (float[12] or NULL) receives every candidate's rate in that order.
 * Results are cached per device and item shapes (ignored when rates is
 * given).  The items' own buffers are not modified.  Synchronises stream.
 */
int dlm_multi_autotune(const dlm_multi_item* items, int32_t count, int32_t calib_iters,
                       dlm_multi_config* best, float* rates, void* stream);

/* ------------------------------------------------------------------------
 * Weighted colouring (WVCP): the iterated feasible/infeasible tabu search of
 * Section 2.2 and Algorithm 2, one workgroup per individual.
 *
 * Round r (r = 0..rounds-1) runs iters_per_round iterations minimising
 * g = (f_w << shift) + phi * c, f_w = sum over classes of the largest weight
 * (eq. (score_WVCP)), c = conflicting edges (eq. (AFISA_score) with phi in
 * fixed point, `shift` fractional bits).  phi_0 = floor(k * max_w * 2^shift /
 * (2 n)); after a round whose best-g state is legal phi is halved, else
 * doubled (at most 2^30); the last round uses phi = (2 max_w) << shift.
 * Moves: every (v, c), c != col v; admissible if v is not frozen or g + delta
 * < best g of the round; choice = lexicographic minimum of (delta g, h, v, c),
 * h = word 0 of Philox(seed; ind, t, v, c), t counting on across rounds; the
 * moved vertex is frozen until t + L + floor(frz_num * n / frz_den), L =
 * floor(w0 * ten_rand / 2^32), w0 = Philox(seed; ind, t, 0, 0x80000001).
 * Each round restarts from the previous round's best-g state.
 *   colors_dev     int16[pop][n]: in = start, out = best legal colouring met
 *                  (or the last round's best-g state if none was legal)
 *   best_legal_dev int32[pop]: its f_w, 0x7fffffff if no legal colouring
 *                  was met, -1 if the start held a colour outside [0, k)
 *   stats_dev      int64[pop][DLM_NSTATS] or NULL: 0 moves, 1 no-ops,
 *                  2 sum deg(v*), 3 tie iterations, 4 rounds whose best-g
 *                  state is legal, 5 final phi
 *   hash_dev       uint64[pop] or NULL: FNV-1a over (v, c, g >> shift)
 * Needs a weighted graph with (2 max_w) << shift <= 2^30, so that every phi
 * fits 31 bits.  Errors: DLM_E_INVAL, DLM_E_UNSUPPORTED (LDS, or weights too
 * large for the shift), DLM_E_HIP.
 * ---------------------------------------------------------------------- */
typedef struct dlm_wvcp_params {
  int32_t k;               /* colours available, 1..32767 */
  int32_t iters_per_round; /* nbIter_TS (10 n in the paper's setting) */
  int32_t rounds;          /* maxLSIters (10) */
  int32_t ten_rand;        /* L uniform in [0, ten_rand), 1..1024 */
  int32_t frz_num;         /* freeze slope numerator (2 for 0.2 |V|) */
  int32_t frz_den;         /* freeze slope denominator (10) */
  int32_t shift;           /* fractional bits of phi, 0..16 (10) */
  int32_t ind_base;        /* global index of row 0 */
  uint64_t seed;           /* Philox key */
  int32_t block;           /* threads per workgroup: 0 = auto, 64, 128, 256 or 512 */
  int32_t reserved;        /* must be 0 */
} dlm_wvcp_params;

int dlm_wvcp_batch(const dlm_graph* g, const dlm_wvcp_params* p, int32_t pop,
                   int16_t* colors_dev, int32_t* best_legal_dev, int64_t* stats_dev,
                   uint64_t* hash_dev, void* stream);

/* ------------------------------------------------------------------------
 * Scores (eq. (f) of Section 2.7 and eq. (score_WVCP) of Section 1).
 *   conflicts_dev int32[count]: monochromatic edges of each colouring
 *   wscore_dev    int32[count] or NULL: sum over colour classes of the largest
 *                 vertex weight (needs a weighted graph)
 * A colouring holding a colour outside [0, k) gets -1 in both outputs.
 * ---------------------------------------------------------------------- */
int dlm_evaluate(const dlm_graph* g, int32_t k, const int16_t* colors_dev, int32_t count,
                 int32_t* conflicts_dev, int32_t* wscore_dev, void* stream);

/* ------------------------------------------------------------------------
 * Greedy partition crossover, GPX (Sections 1 and 2.6: the offspring
 * inherits alternately the largest remaining colour class of each parent;
 * the crossover is asymmetric, the individual being the first parent).
 * Child j of pair p (child id c = child_base + p * per_pair + j) is built
 * from A = parents[pairs[p][0]] (first) and B = parents[pairs[p][1]]: step
 * l = 0..k-1 takes A when l is even and B when l is odd, picks the class of
 * that parent with the most still-unassigned vertices (ties: smallest word 0
 * of Philox(seed; c, l, u, 0x80000007) with u the lowest unassigned vertex
 * of the class, then smallest u) and gives its unassigned vertices colour l.
 * Vertices left after k steps get floor(w0 * k / 2^32), w0 =
 * Philox(seed; c, 0, v, 0x80000003).
 *   parents_dev  int16[pop][n], colours in [0, k)
 *   pairs_dev    int32[npairs][2], indices in [0, pop)
 *   children_dev int16[npairs * per_pair][n] output; a child whose pair
 *                index or parent colour is out of range is all -1
 * ---------------------------------------------------------------------- */
int dlm_gpx_batch(const dlm_graph* g, int32_t k, const int16_t* parents_dev, int32_t pop,
                  const int32_t* pairs_dev, int32_t npairs, int32_t per_pair, uint64_t seed,
                  uint32_t child_base, int16_t* children_dev, void* stream);

/* ------------------------------------------------------------------------
 * Offspring selection (eq. (select_cross) of Section 2.6 taken
 * population-wide): keep `keep` of `count` candidates.
 *   DLM_SELECT_TOP (learned loop): the smallest predicted scores, ties by
 *     index (NaN ranks last);
 *   DLM_SELECT_RANDOM (plain loop): the smallest word 0 of
 *     Philox(seed; i, gen, 0, 0x80000006), ties by index; scores unused.
 *   scores_dev   float[count] (may be NULL in random mode)
 *   idx_out_dev  int32[keep] output: selected indices in rank order
 *   workspace_dev  caller-owned scratch of 8 * count bytes
 * ---------------------------------------------------------------------- */
#define DLM_SELECT_TOP 0
#define DLM_SELECT_RANDOM 1
int dlm_select(const float* scores_dev, int32_t count, int32_t keep, int32_t mode, uint64_t seed,
               uint32_t gen, int32_t* idx_out_dev, void* workspace_dev, void* stream);

/* ------------------------------------------------------------------------
 * Device steps of one memetic generation (Algorithm 1) in the simplified
 * form of this library: random partner pairing, offspring gather, target
 * standardisation for the scorer, and the (mu + lambda) population update
 * that stands in for the paper's distance-based update (Section 2.5).
 * ---------------------------------------------------------------------- */

/* dst[r] = src[idx[r]] for r < count (rows of n int16); a row whose index is
 * outside [0, rows) is filled with -1. */
int dlm_gather_rows(const int16_t* src_dev, int32_t rows, int32_t n, const int32_t* idx_dev,
                    int32_t count, int16_t* dst_dev, void* stream);

/* out[i] = (f[i] - mean) / std over the count values (FP64 statistics,
 * population standard deviation; all zero if std = 0): the scorer's
 * training targets for one generation. */
int dlm_standardize(const int32_t* f_dev, int32_t count, float* out_dev, void* stream);

/* Training scores of one WVCP generation (Section 2.3 trains on the
 * post-search score; a search that met no legal colouring, score
 * 0x7fffffff, takes the worst legal score of the generation):
 * out_dev[i] = f_dev[i] if legal, else max over the legal f_dev; the
 * device int *any_legal_dev is set to 1 if some f_dev[i] is legal, else 0
 * (out_dev is then a copy of f_dev and the generation trains nothing).
 * count >= 1; out_dev may equal f_dev.  Asynchronous on stream. */
int dlm_wvcp_targets(const int32_t* f_dev, int32_t count, int32_t* out_dev, int32_t* any_legal_dev, void* stream);

/* pairs_dev int32[pop][2] = (i, j): j uniform over the other members,
 * j = floor(w0 (pop - 1) / 2^32) + (that value >= i), w0 = word 0 of
 * Philox(seed; i, gen, 0, 0x80000009). */
int dlm_random_pairs(int32_t pop, uint64_t seed, uint32_t gen, int32_t* pairs_dev, void* stream);

/* One offspring per individual (eq. select_cross with K-nearest matching,
 * Section 2.6): idx_dev[g] = gK + j for the child j < K of group g (children
 * gK .. gK + K - 1) with the smallest FP32 score, ties by smaller j
 * (DLM_SELECT_TOP), or j = floor(w0 K / 2^32), w0 = word 0 of
 * Philox(seed; g, gen, 0, 0x8000000A) (DLM_SELECT_RANDOM, scores unused). */
int dlm_select_groups(const float* scores_dev, int32_t groups, int32_t K, int32_t mode, uint64_t seed,
                      uint32_t gen, int32_t* idx_dev, void* stream);

/* The step from k to k - 1 colours of the decreasing-k driver (Section
 * 2.7: once a legal k-colouring is found, k drops by one), in place on
 * colors_dev (int16 [pop][n]): each row's smallest class (ties by smaller
 * colour) is dissolved, its vertex v takes colour floor(w0 (k - 1) / 2^32),
 * w0 = word 0 of Philox(seed; row, step, v, 0x8000000B), and colours above
 * the dissolved one move down by one.  A row with a colour outside [0, k)
 * becomes all -1.  2 <= k <= 32767, n <= 32767. */
int dlm_reduce_colours(int16_t* colors_dev, int32_t pop, int32_t n, int32_t k, uint64_t seed, uint32_t step,
                       void* stream);

/* Keep the pop best of parents (indices 0..pop-1) and offspring (indices
 * pop..2pop-1) by score ascending, ties by index: out_dev int16[pop][n] and
 * f_out_dev int32[pop] in rank order.  workspace_dev: 24 * pop bytes. */
int dlm_pop_update(const int16_t* parents_dev, const int32_t* f_parents_dev,
                   const int16_t* offspring_dev, const int32_t* f_offspring_dev, int32_t pop,
                   int32_t n, int16_t* out_dev, int32_t* f_out_dev, void* workspace_dev,
                   void* stream);

/* ------------------------------------------------------------------------
 * Distance-based population management (Sections 2.4 to 2.6): the
 * approximate partition distance, the population update under a minimum
 * spacing, and the K nearest neighbours for parent matching.  A pool's
 * distances live in one int32 matrix (row stride ld); the update and the
 * gather read only its strict upper triangle, so the blocks of a new
 * generation can be written straight into it (old x new by the block form,
 * new x new by the triangle form, old x old gathered from the last pool).
 * ---------------------------------------------------------------------- */

/* Approximate set-theoretic partition distance (Section 2.4) of every pair
 * (row i of a, row j of b):
 *   M[c][d] = |{v : a_i[v] = c and b_j[v] = d}|;
 *   S_ab: the classes of a_i by decreasing size (ties by index) each take the
 *         free class of b_j with the largest positive M (ties by index);
 *   S_ba: the same with a_i and b_j swapped;
 *   out_dev[i * ld + j] = n - max(S_ab, S_ba).
 * An upper bound of the exact distance (n - a maximum matching on M), equal
 * to it on close partitions.
 *   a_dev, b_dev  int16 device colourings [na][n], [nb][n], colours in [0, k);
 *                 a pair with a colour outside [0, k) gets -1
 *   tri           0: all na x nb pairs; 1: a_dev == b_dev and na == nb, the
 *                 pairs i < j, mirrored below the diagonal, diagonal 0;
 *                 2: as 1 without the mirror (the strict lower triangle is
 *                 not written), the form a pool matrix needs
 *   out_dev       int32, row stride ld >= nb elements
 *   workspace_dev caller-owned scratch of 2 (k + 2) (na + nb) bytes (the
 *                 class orders)
 * 1 <= n <= 32767, 1 <= k <= 256.  DLM_E_INVAL on bad sizes or null buffers. */
int dlm_partition_distance(int32_t n, int32_t k, const int16_t* a_dev, int32_t na, const int16_t* b_dev,
                           int32_t nb, int32_t tri, int32_t* out_dev, int64_t ld, void* workspace_dev,
                           void* stream);

/* Distance-and-quality population update (Section 2.5).  The pool is fa
 * (indices 0..na-1) then fb (na..na+nb-1), lower score better.  Taken in
 * order of (score, index), a member joins when its distance to every
 * member already taken is > spacing (the paper's |V| / 10); if the pool
 * runs out first, the best members left out fill the places.
 *   dist_dev      int32 pool distances; only [lo * ld + hi], lo < hi, is read
 *   pick_dev      int32 [keep] output: pool indices in the order taken
 *   n_spaced_dev  int32 [1] output: how many were taken under the spacing
 *   workspace_dev caller-owned scratch of 4 (na + nb) bytes
 * na + nb <= 65536, 0 <= keep <= na + nb, ld >= na + nb.  The walk goes in
 * chunks of 512 members: many workgroups check a chunk against the members
 * taken before it, then one workgroup settles the chunk in order; the result
 * is that of the one-at-a-time walk.  n_spaced_dev also carries the running
 * count between the chunks, so it must not alias another argument. */
int dlm_spacing_update(const int32_t* fa_dev, int32_t na, const int32_t* fb_dev, int32_t nb,
                       const int32_t* dist_dev, int64_t ld, int32_t keep, int32_t spacing,
                       int32_t* pick_dev, int32_t* n_spaced_dev, void* workspace_dev, void* stream);

/* out_dev[a * ld_out + b] = dist_dev[lo * ld + hi], lo / hi the smaller /
 * larger of idx[a], idx[b], and 0 for a = b: the distances of the members a
 * pick keeps, as a full symmetric count x count matrix. */
int dlm_gather_distances(const int32_t* dist_dev, int64_t ld, const int32_t* idx_dev, int32_t count,
                         int32_t* out_dev, int64_t ld_out, void* stream);

/* Rows and scores of picked pool members: row r of out_dev (int16 [count][n])
 * and fout_dev[r] come from member pick[r] (a row of ra_dev / fa_dev below
 * na, else of rb_dev / fb_dev); an index outside [0, na + nb) gives a row of
 * -1 and score -1. */
int dlm_gather_pool(const int16_t* ra_dev, const int32_t* fa_dev, int32_t na, const int16_t* rb_dev,
                    const int32_t* fb_dev, int32_t nb, int32_t n, const int32_t* pick_dev, int32_t count,
                    int16_t* out_dev, int32_t* fout_dev, void* stream);

/* K-nearest-neighbour parent matching (Section 2.6): nn_dev[i * K + t] is
 * the t-th nearest j != i by dist_dev[i * ld + j] (a full symmetric p x p
 * matrix), ties by smaller j.  0 <= K <= p - 1, p <= 65536, distances in
 * [0, 65535]. */
int dlm_nearest(const int32_t* dist_dev, int64_t ld, int32_t p, int32_t K, int32_t* nn_dev, void* stream);

/* ------------------------------------------------------------------------
 * Offspring scorer (Section 2.3): a colour-permutation-invariant regressor
 * of the post-search score, trained online with Adam on (start colouring,
 * score after tabu search) pairs, and used by eq. (select_cross) to rank
 * offspring.  Form: shared per-class MLP over the class indicator vectors V_i,
 * sum pooling over the k classes, small head:
 *   h1_i = LReLU(b1 + V_i W1)  [H1]     h2_i = LReLU(b2 + h1_i W2)  [H2]
 *   z = sum_i h2_i              h3 = LReLU(b3 + z W3)  [H3]
 *   y = h3 . w4 + b4            LReLU(x) = max(0.2 x, x)
 * Only (H1, H2, H3) = (256, 128, 64) is built.  Layer 1 is a gather of W1
 * rows (equal to the indicator product); layer 2 and its backward products
 * use BF16 MFMA with FP32 accumulation; FP32 master weights and Adam state,
 * a BF16 working copy of W2 (layer 1 gathers the FP32 W1 rows).  All
 * reductions run in a fixed order, so results are deterministic.
 *
 * params_host: FP32, packed W1 [n][H1], b1 [H1], W2 [H1][H2], b2 [H2],
 * W3 [H2][H3], b3 [H3], w4 [H3], b4 [1] (row-major); copied at creation.
 * max_batch bounds the batch of dlm_scorer_train / dlm_scorer_grad (the
 * scorer allocates its training activations for that size).  k <= 256.
 * ---------------------------------------------------------------------- */
typedef struct dlm_scorer dlm_scorer; /* opaque: weights, Adam state, workspace */

int dlm_scorer_create(int32_t n, int32_t k, int32_t h1, int32_t h2, int32_t h3, int32_t max_batch,
                      const float* params_host, dlm_scorer** out);
int dlm_scorer_destroy(dlm_scorer* s);
/* number of FP32 parameters (the packed layout above) */
int dlm_scorer_num_params(const dlm_scorer* s, int64_t* count);
/* copy the FP32 master parameters (packed layout) to params_dev */
int dlm_scorer_get_params(const dlm_scorer* s, float* params_dev, void* stream);

/*
 * Predict the post-search score of `count` colourings.
 *   colors_dev int16[count][n], colours in [0, k)
 *   scores_dev float[count] output
 * Not safe to run concurrently with dlm_scorer_train on the same scorer.
 */
int dlm_score_offspring(const dlm_scorer* s, const int16_t* colors_dev, int32_t count,
                        float* scores_dev, void* stream);

/*
 * Gradient of the mean squared error (1/count) sum_b (y_b - t_b)^2 with
 * respect to the packed parameters (1 <= count <= max_batch), written to
 * grad_dev (float[num_params], may be NULL); loss_dev (float[1], may be NULL)
 * receives the loss.  The parameters are not changed.
 */
int dlm_scorer_grad(dlm_scorer* s, const int16_t* colors_dev, const float* targets_dev,
                    int32_t count, float* grad_dev, float* loss_dev, void* stream);

/*
 * Online training (Section 2.3): `epochs` passes over the `count` pairs in
 * consecutive mini-batches of `batch` (the last may be smaller); each
 * mini-batch is one Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias
 * correction counted over the scorer's lifetime) on the FP32 master weights,
 * followed by a BF16 re-cast.  loss_dev (float[epochs * ceil(count/batch)],
 * may be NULL) receives each step's loss before its update.
 */
int dlm_scorer_train(dlm_scorer* s, const int16_t* colors_dev, const float* targets_dev,
                     int32_t count, int32_t batch, int32_t epochs, float lr, float* loss_dev,
                     void* stream);

/* ------------------------------------------------------------------------
 * The paper's colour-invariant network (Section 2.3) as a scorer: a
 * colouring S = (V_1 .. V_k) enters as its k class indicator vectors over
 * the n vertices; layer j maps the k class rows X_i (width l_in) to
 *   Z_i = X_i Lambda_j + rho(X) Gamma_j + beta_j,  rho(X) = (1/k) sum_i X_i
 * hidden layers: X'_i = LReLU_0.2(BN(Z)_i), with the invariant batch
 * normalisation over the batch and all k classes per feature (eps 1e-5,
 * learnable scale gamma_j and shift mu_j per feature, running estimates with
 * momentum 0.1 and the unbiased variance); the last layer has width 1 and
 * the output is (1/k) sum_i Z_i.  The hidden layers' products are GEMMs with
 * BF16 operands and FP32 accumulation (dlm_gemm_bf16); the output layer's products
 * and everything else run in FP32 on kernels of this library, reductions in
 * a fixed order.
 *
 * widths: nl layer widths (hidden ..., 1).  params_host: FP32, per layer
 * Lambda [l_in][l_out], Gamma [l_in][l_out], beta [l_out], then for hidden
 * layers gamma [l_out], mu [l_out] (row-major; the trainables), followed by
 * the running mean [l_out] and running variance [l_out] of every hidden layer
 * in order; copied at creation.  max_batch bounds the colourings of one
 * training step and the chunk of one evaluation pass; the network allocates
 * its activations for that many (about 6 (max_batch k) sum(widths) + 6
 * (max_batch k) n bytes).  2 <= k <= 32767, n <= 32767, max_batch <= 65535,
 * max_batch k < 2^31.
 * ---------------------------------------------------------------------- */
/* Calls on one network share its activation buffers and streams:
 * they must not overlap (one stream, or ordered by the caller).  Each call
 * is ordered on the stream it is given: the network's second stream forks
 * from it and joins it again before the call returns.  Use a network on the
 * device that was current at its creation.  Errors return a
 * negative code with a message from dlm_last_error(); device buffers belong
 * to the caller, the network owns its own memory until dlm_invnet_destroy. */
typedef struct dlm_invnet dlm_invnet; /* opaque: weights, Adam state, activations, second stream */

int dlm_invnet_create(int32_t n, int32_t k, int32_t nl, const int32_t* widths, const float* params_host,
                      int32_t max_batch, dlm_invnet** out);
int dlm_invnet_destroy(dlm_invnet* s);
/* sizes of the two parts of the packed layout above */
int dlm_invnet_num_params(const dlm_invnet* s, int64_t* trainable, int64_t* running);
/* copy the FP32 trainables, then the running estimates (packed layout), to params_dev */
int dlm_invnet_get_params(const dlm_invnet* s, float* params_dev, void* stream);

/*
 * Evaluation: out_dev[c] = f(colouring c) for `count` colourings
 * (colors_dev int16[count][n], colours in [0, k)), the normalisation taken
 * from the running estimates; chunks of max_batch.  A colour outside [0, k)
 * gives that vertex no class.
 */
int dlm_invnet_forward(dlm_invnet* s, const int16_t* colors_dev, int32_t count, float* out_dev, void* stream);

/*
 * Gradient of the mean squared error (1/count) sum_c (f_c - t_c)^2 on one
 * batch (1 <= count <= max_batch), the normalisation from the batch's own
 * statistics, written to grad_dev (float[trainable], may be NULL); loss_dev
 * (float[1], may be NULL) receives the loss.  Neither the trainables nor the
 * running estimates change.
 */
int dlm_invnet_grad(dlm_invnet* s, const int16_t* colors_dev, const float* targets_dev, int32_t count,
                    float* grad_dev, float* loss_dev, void* stream);

/*
 * Training: `epochs` passes over the `count` pairs in consecutive batches of
 * `batch` (the last may be smaller); each batch is a training-mode forward
 * (which also moves the running estimates), the MSE gradient and one Adam
 * step (beta1 0.9, beta2 0.999, eps 1e-8, bias correction counted over the
 * network's lifetime) on the FP32 trainables, then a BF16 re-cast of every
 * Lambda and Gamma.  loss_dev (float[epochs * ceil(count/batch)], may be
 * NULL) receives each step's loss before its update.
 */
int dlm_invnet_train(dlm_invnet* s, const int16_t* colors_dev, const float* targets_dev, int32_t count,
                     int32_t batch, int32_t epochs, float lr, float* loss_dev, void* stream);

/*
 * The network's matrix product on its own (Section 2.3: the layer products
 * X Lambda and R Gamma, their weight gradients X^T dZ and input gradients
 * dZ Lambda^T), exposed so that it can be checked and timed alone:
 *   C[m][n] = sum_{k < K} A(m, k) B(k, n)   for m < M, n < N,
 * A(m, k) = A_dev[m sa + k] if a_kcontig else A_dev[k sa + m],
 * B(k, n) = B_dev[n sb + k] if b_kcontig else B_dev[k sb + n],
 * A and B BF16 (raw 16-bit patterns), C FP32 row-major with pitch ldc >= N;
 * products accumulate in FP32 (MFMA 32x32x16).  K = 0 writes zeros; M or
 * N = 0 does nothing.  Any pitch and alignment work; pitches and pointers
 * that are multiples of 4 values (8 bytes) read fastest.
 * tile: 0 picks the workgroup tile (64, 128 or 256 square) from the shape,
 * else that tile.  splits: 0 picks from the shape whether to cut K into
 * chunks (when the tile grid is too small to fill the device), else that
 * many chunks; chunk s writes its partial product into workspace_dev
 * (float[splits][M][N], caller-owned, used only when splits > 1 and it is
 * large enough; may be NULL) and a second kernel adds the partials in chunk
 * order.  The result depends only on the shape, the tile and the split, so
 * repeated calls give identical bits.  Errors: negative sizes, ldc < N, a
 * pitch smaller than its contiguous extent, a bad tile, a forced split
 * without room, or a null operand.  Asynchronous on stream.
 */
int dlm_gemm_bf16(int32_t a_kcontig, const uint16_t* A_dev, int64_t sa, int32_t b_kcontig, const uint16_t* B_dev,
                  int64_t sb, float* C_dev, int64_t ldc, int32_t M, int32_t N, int32_t K, int32_t tile,
                  int32_t splits, void* workspace_dev, int64_t workspace_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Measurement helper (not part of the search): sustained LDS read bandwidth
 * of the whole device in bytes/s, from a kernel that streams conflict-free
 * 16-byte LDS reads on every resident workgroup for `rounds` passes over a
 * 64 KiB buffer.  It is the measured denominator of the TabuCol kernel's LDS
 * roofline.  Synchronises stream.
 * ---------------------------------------------------------------------- */
int dlm_probe_lds_bandwidth(int32_t rounds, double* bytes_per_s, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* DLMCOL_H */
