/*
 * CPU oracle for the population graph-coloring hot path of the deep-learning
 * guided memetic coloring method (Goudet, Grelier and Hao, "A deep learning
 * guided memetic framework for graph coloring problems").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant
 * generator with the HIP kernels: both sides implement the same written
 * conventions independently.
 *
 * Plain, slow and obviously correct: every function follows one passage of
 * the paper, or a plain definition, step by step in the paper's order.
 *
 *   conflicts()         eq. (f), Section 2.7: number of monochromatic edges.
 *   wscore()            eq. (score_WVCP), Section 1: sum over colour classes
 *                       of the largest vertex weight in the class.
 *   orc_init_random()   Section 2.7: each vertex gets a uniform colour.
 *   orc_greedy_init()   Section 2.1: randomized greedy WVCP initialisation.
 *   orc_tabucol()       Section 2.7: TabuCol (Hertz and de Werra, with the
 *                       Galinier-Hao gamma table) run for a fixed budget.
 *   orc_wvcp_tabu()     Section 2.2, eq. (AFISA_score), Algorithm 2: the
 *                       iterated feasible/infeasible tabu search with the
 *                       adaptive penalty phi and vertex freezing.
 *   orc_gpx()           Sections 1 and 2.6: greedy partition crossover.
 *   orc_select()        Section 2.6, eq. (select_cross): keep the offspring
 *                       with the best predicted score (population-wide
 *                       top-`keep` reading), or a random subset for the
 *                       plain loop.
 *
 * Conventions the paper leaves open (both sides follow them):
 *   Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11) keyed by the 64-bit
 *   seed (k0 = low word, k1 = high word); counters:
 *     tie hash         (ind, t, v, c)
 *     tenure random L  (ind, t, 0, 0x80000001)
 *     random init      (ind, 0, v, 0x80000002)
 *     GPX leftovers    (child, 0, v, 0x80000003)
 *     selection        (i, gen, 0, 0x80000006)
 *     GPX class ties   (child, step, min vertex of class, 0x80000007)
 *     greedy init pick (ind, 0, v, 0x80000008)
 *   Uniform integer in [0, K): (w0 * K) >> 32 (Lemire, no rejection).
 *   Tabu tenure (COL): L + min(floor(num * f_after / den), 32757), L uniform
 *   in [0, ten_rand); the pair (v, old colour) is tabu while t < t_move + tt.
 *   Aspiration: a tabu move is allowed when f + delta < f_best of the call.
 *   Move choice: lexicographic minimum of (delta, hash, v, c) over the
 *   admissible one-moves of conflicting vertices; none admissible => the
 *   iteration is a no-op.
 *
 * Parity pins: see the test suite (closed forms, brute force on tiny graphs,
 * invariants checked every iteration in check mode).
 */
#include <limits.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define D_TENURE 0x80000001u
#define D_INIT 0x80000002u
#define D_GPXFILL 0x80000003u
#define D_SELECT 0x80000006u
#define D_GPXTIE 0x80000007u
#define D_GREEDY 0x80000008u

#define TT_CAP 32757
#define ORC_NSTATS 8

static char orc_err[512];

const char* orc_last_error(void) { return orc_err; }

/* ------------------------------------------------------------------ */
/* Philox4x32-10, written from the SC'11 definition.                   */
/* ------------------------------------------------------------------ */
void orc_philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint64_t seed,
                uint32_t out[4]) {
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  uint32_t x0 = c0, x1 = c1, x2 = c2, x3 = c3;
  for (int r = 0; r < 10; r++) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    uint32_t y3 = lo0;
    x0 = y0;
    x1 = y1;
    x2 = y2;
    x3 = y3;
  }
  out[0] = x0;
  out[1] = x1;
  out[2] = x2;
  out[3] = x3;
}

static uint32_t word0(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint64_t seed) {
  uint32_t o[4];
  orc_philox(c0, c1, c2, c3, seed, o);
  return o[0];
}

uint32_t orc_uniform(uint32_t x, uint32_t K) { return (uint32_t)(((uint64_t)x * K) >> 32); }

/* ------------------------------------------------------------------ */
/* Plain definitions: conflicts (eq. f) and weighted score.            */
/* ------------------------------------------------------------------ */
int64_t orc_conflicts(int32_t n, const int32_t* rp, const int32_t* ci, const int16_t* col) {
  int64_t f = 0;
  for (int32_t u = 0; u < n; u++)
    for (int32_t e = rp[u]; e < rp[u + 1]; e++) {
      int32_t v = ci[e];
      if (u < v && col[u] == col[v]) f++;
    }
  return f;
}

/* sum over non-empty colour classes of the largest weight in the class */
int64_t orc_wscore(int32_t n, const int32_t* w, int32_t k, const int16_t* col) {
  int64_t* mx = (int64_t*)calloc((size_t)k, sizeof(int64_t));
  for (int32_t v = 0; v < n; v++)
    if (w[v] > mx[col[v]]) mx[col[v]] = w[v];
  int64_t s = 0;
  for (int32_t c = 0; c < k; c++) s += mx[c];
  free(mx);
  return s;
}

/* ------------------------------------------------------------------ */
/* Initialisation.                                                     */
/* ------------------------------------------------------------------ */
void orc_init_random(int32_t n, int32_t k, int32_t pop, uint64_t seed, int32_t ind_base,
                     int16_t* colors) {
  for (int32_t i = 0; i < pop; i++)
    for (int32_t v = 0; v < n; v++)
      colors[(int64_t)i * n + v] =
          (int16_t)orc_uniform(word0((uint32_t)(ind_base + i), 0, (uint32_t)v, D_INIT, seed),
                               (uint32_t)k);
}

/*
 * Section 2.1: vertices by weight descending, then degree descending (then
 * index ascending); each takes a random already-used colour that creates no
 * conflict, else a new colour.  Colours are numbered in creation order.
 * Returns the number of colours used.
 */
int32_t orc_greedy_init(int32_t n, const int32_t* rp, const int32_t* ci, const int32_t* w,
                        uint64_t seed, int32_t ind, int16_t* col) {
  int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  for (int32_t v = 0; v < n; v++) order[v] = v;
  /* insertion sort by (w desc, deg desc, index asc): plain and stable */
  for (int32_t a = 1; a < n; a++) {
    int32_t x = order[a], b = a - 1;
    while (b >= 0) {
      int32_t y = order[b];
      int32_t dx = rp[x + 1] - rp[x], dy = rp[y + 1] - rp[y];
      int before = (w[x] > w[y]) || (w[x] == w[y] && dx > dy) ||
                   (w[x] == w[y] && dx == dy && x < y);
      if (!before) break;
      order[b + 1] = y;
      b--;
    }
    order[b + 1] = x;
  }
  for (int32_t v = 0; v < n; v++) col[v] = -1;
  int32_t used = 0;
  unsigned char* blocked = (unsigned char*)calloc((size_t)n + 1, 1);
  int32_t* feas = (int32_t*)malloc(sizeof(int32_t) * ((size_t)n + 1));
  for (int32_t a = 0; a < n; a++) {
    int32_t v = order[a];
    memset(blocked, 0, (size_t)used + 1);
    for (int32_t e = rp[v]; e < rp[v + 1]; e++) {
      int32_t u = ci[e];
      if (col[u] >= 0) blocked[col[u]] = 1;
    }
    int32_t nf = 0;
    for (int32_t c = 0; c < used; c++)
      if (!blocked[c]) feas[nf++] = c;
    if (nf > 0) {
      uint32_t r = orc_uniform(word0((uint32_t)ind, 0, (uint32_t)v, D_GREEDY, seed), (uint32_t)nf);
      col[v] = (int16_t)feas[r];
    } else {
      col[v] = (int16_t)used;
      used++;
    }
  }
  free(order);
  free(blocked);
  free(feas);
  return used;
}

/* ------------------------------------------------------------------ */
/* Trajectory fingerprint (FNV-1a over 64-bit move records).           */
/* ------------------------------------------------------------------ */
#define FNV_OFF 0xcbf29ce484222325ull
#define FNV_PRIME 0x100000001b3ull
static uint64_t fnv_step(uint64_t h, uint32_t v, uint32_t c, int64_t f) {
  uint64_t x = (uint64_t)(v & 0xffffu) | ((uint64_t)(c & 0xffffu) << 16) |
               ((uint64_t)(uint32_t)f << 32);
  return (h ^ x) * FNV_PRIME;
}

/* lexicographic order on (delta, hash, v, c); hash evaluated on demand */
typedef struct {
  int64_t d;
  int has_h;
  uint32_t h;
  int32_t v, c;
} cand_t;

static int cand_better(cand_t* a, cand_t* b, uint64_t seed, uint32_t ind, uint32_t t) {
  /* is a strictly smaller than b?  b->v < 0 means "no candidate" */
  if (b->v < 0) return 1;
  if (a->d != b->d) return a->d < b->d;
  if (!a->has_h) {
    a->h = word0(ind, t, (uint32_t)a->v, (uint32_t)a->c, seed);
    a->has_h = 1;
  }
  if (!b->has_h) {
    b->h = word0(ind, t, (uint32_t)b->v, (uint32_t)b->c, seed);
    b->has_h = 1;
  }
  if (a->h != b->h) return a->h < b->h;
  if (a->v != b->v) return a->v < b->v;
  return a->c < b->c;
}

/* ------------------------------------------------------------------ */
/* TabuCol (Section 2.7).                                              */
/* ------------------------------------------------------------------ */
typedef struct {
  int32_t k, max_iters, ten_num, ten_den, ten_rand, check;
  uint64_t seed;
} orc_tabu_params;

/*
 * One individual.  colors: in = start colouring S^O, out = best colouring
 * S' met on the trajectory.  stats[ORC_NSTATS]:
 *   0 moves, 1 no-op iterations, 2 sum over iterations of the number of
 *   conflicting vertices scanned, 3 sum over moves of deg(v*), 4 iterations
 *   whose minimum delta was shared by >= 2 admissible moves, 5 tenure-cap hits.
 * trace (optional, trace_cap records): {v | c << 16, f after the move};
 * a no-op records v = c = 0xffff.
 * Returns 0, or -1 when check mode finds a broken invariant.
 */
int orc_tabucol(int32_t n, const int32_t* rp, const int32_t* ci, const orc_tabu_params* p,
                int32_t ind, int16_t* colors, int32_t* f_best_out, int32_t* iters_out,
                int64_t* stats, uint64_t* hash_out, int32_t* trace, int32_t trace_cap) {
  const int32_t k = p->k;
  int16_t* col = (int16_t*)malloc(sizeof(int16_t) * (size_t)n);
  int16_t* best = (int16_t*)malloc(sizeof(int16_t) * (size_t)n);
  int32_t* gamma = (int32_t*)calloc((size_t)n * k, sizeof(int32_t));
  int64_t* tabu = (int64_t*)calloc((size_t)n * k, sizeof(int64_t));
  int rc = 0;
  memcpy(col, colors, sizeof(int16_t) * (size_t)n);
  for (int s = 0; s < ORC_NSTATS; s++) stats[s] = 0;

  /* gamma[v][c] = number of neighbours of v coloured c */
  for (int32_t v = 0; v < n; v++)
    for (int32_t e = rp[v]; e < rp[v + 1]; e++) gamma[(int64_t)v * k + col[ci[e]]]++;
  int64_t f = 0;
  for (int32_t v = 0; v < n; v++) f += gamma[(int64_t)v * k + col[v]];
  f /= 2;
  int64_t f_best = f;
  memcpy(best, col, sizeof(int16_t) * (size_t)n);
  uint64_t h = FNV_OFF;
  int64_t t = 0;
  const uint32_t uind = (uint32_t)ind;

  while (t < p->max_iters && f > 0) {
    /* scan: one-moves of conflicting vertices */
    cand_t bestc;
    bestc.v = -1;
    bestc.has_h = 0;
    int64_t nconf = 0, nmin = 0;
    for (int32_t v = 0; v < n; v++) {
      int32_t cv = col[v];
      int32_t gcur = gamma[(int64_t)v * k + cv];
      if (gcur == 0) continue;
      nconf++;
      for (int32_t c = 0; c < k; c++) {
        if (c == cv) continue;
        int64_t d = (int64_t)gamma[(int64_t)v * k + c] - gcur;
        int tabu_now = tabu[(int64_t)v * k + c] > t;
        if (tabu_now && !(f + d < f_best)) continue;
        cand_t cc = {d, 0, 0, v, c};
        if (bestc.v >= 0 && d == bestc.d) nmin++;
        else if (bestc.v < 0 || d < bestc.d) nmin = 1;
        if (cand_better(&cc, &bestc, p->seed, uind, (uint32_t)t)) bestc = cc;
      }
    }
    stats[2] += nconf;
    if (nmin >= 2) stats[4]++;

    if (p->check) {
      /* independent re-derivation of the choice from the colours alone */
      cand_t bc = {0, 0, 0, -1, -1};
      int64_t frec = orc_conflicts(n, rp, ci, col);
      if (frec != f) {
        snprintf(orc_err, sizeof orc_err, "ind %d t %lld: f=%lld recount=%lld", ind,
                 (long long)t, (long long)f, (long long)frec);
        rc = -1;
        break;
      }
      for (int32_t v = 0; v < n; v++) {
        int32_t same = 0;
        for (int32_t e = rp[v]; e < rp[v + 1]; e++) same += col[ci[e]] == col[v];
        for (int32_t c = 0; c < k; c++) {
          int32_t g = 0;
          for (int32_t e = rp[v]; e < rp[v + 1]; e++) g += col[ci[e]] == c;
          if (g != gamma[(int64_t)v * k + c]) {
            snprintf(orc_err, sizeof orc_err, "ind %d t %lld: gamma[%d][%d]=%d recount=%d", ind,
                     (long long)t, v, c, gamma[(int64_t)v * k + c], g);
            rc = -1;
          }
          if (same == 0 || c == col[v]) continue;
          int64_t d = (int64_t)g - same;
          if (tabu[(int64_t)v * k + c] > t && !(f + d < f_best)) continue;
          cand_t cc = {d, 1, word0(uind, (uint32_t)t, (uint32_t)v, (uint32_t)c, p->seed), v, c};
          int better = bc.v < 0 || cc.d < bc.d ||
                       (cc.d == bc.d && (cc.h < bc.h || (cc.h == bc.h && (cc.v < bc.v ||
                                                                         (cc.v == bc.v && cc.c < bc.c)))));
          if (better) bc = cc;
        }
      }
      if (rc) break;
      if (bc.v != bestc.v || (bc.v >= 0 && bc.c != bestc.c)) {
        snprintf(orc_err, sizeof orc_err, "ind %d t %lld: chosen (%d,%d) brute (%d,%d)", ind,
                 (long long)t, bestc.v, bestc.c, bc.v, bc.c);
        rc = -1;
        break;
      }
    }

    if (bestc.v < 0) { /* nothing admissible: no-op iteration */
      stats[1]++;
      h = fnv_step(h, 0xffffu, 0xffffu, f);
      if (trace && t < trace_cap) {
        trace[2 * t] = (int32_t)0xffffffffu;
        trace[2 * t + 1] = (int32_t)f;
      }
      t++;
      continue;
    }

    /* apply the move (v*, c*) */
    const int32_t v = bestc.v, c = bestc.c, old = col[v];
    col[v] = (int16_t)c;
    for (int32_t e = rp[v]; e < rp[v + 1]; e++) {
      int32_t u = ci[e];
      gamma[(int64_t)u * k + old]--;
      gamma[(int64_t)u * k + c]++;
    }
    f += bestc.d;
    int64_t tt_f = (int64_t)p->ten_num * f / p->ten_den;
    if (tt_f > TT_CAP) {
      tt_f = TT_CAP;
      stats[5]++;
    }
    int64_t L = orc_uniform(word0(uind, (uint32_t)t, 0, D_TENURE, p->seed), (uint32_t)p->ten_rand);
    tabu[(int64_t)v * k + old] = t + L + tt_f;
    if (f < f_best) {
      f_best = f;
      memcpy(best, col, sizeof(int16_t) * (size_t)n);
    }
    stats[0]++;
    stats[3] += rp[v + 1] - rp[v];
    h = fnv_step(h, (uint32_t)v, (uint32_t)c, f);
    if (trace && t < trace_cap) {
      trace[2 * t] = (v & 0xffff) | (c << 16);
      trace[2 * t + 1] = (int32_t)f;
    }
    t++;
  }
  memcpy(colors, best, sizeof(int16_t) * (size_t)n);
  *f_best_out = (int32_t)f_best;
  *iters_out = (int32_t)t;
  *hash_out = h;
  free(col);
  free(best);
  free(gamma);
  free(tabu);
  return rc;
}

/* Many independent individuals (rows of `colors` belong to ind_ids[i]). */
int orc_tabucol_batch(int32_t n, const int32_t* rp, const int32_t* ci, const orc_tabu_params* p,
                      int32_t count, const int32_t* ind_ids, int16_t* colors, int32_t* f_best,
                      int32_t* iters, int64_t* stats, uint64_t* hashes, int32_t nthreads) {
  int rc = 0;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads) reduction(| : rc)
  for (int32_t i = 0; i < count; i++) {
    int r = orc_tabucol(n, rp, ci, p, ind_ids[i], colors + (int64_t)i * n, f_best + i, iters + i,
                        stats + (int64_t)i * ORC_NSTATS, hashes + i, NULL, 0);
    rc |= (r != 0);
  }
  return rc ? -1 : 0;
}

/* ------------------------------------------------------------------ */
/* Weighted colouring: iterated feasible/infeasible tabu (Section 2.2). */
/* ------------------------------------------------------------------ */
typedef struct {
  int32_t k, iters_per_round, rounds, ten_rand, frz_num, frz_den, shift, check;
  uint64_t seed;
} orc_wvcp_params;

/* class statistics: largest weight, how many vertices hold it, second largest */
typedef struct {
  int64_t m1, cnt1, m2;
} cls_t;

static void class_stats(int32_t n, const int32_t* w, const int16_t* col, int32_t c, cls_t* s) {
  s->m1 = 0;
  s->cnt1 = 0;
  s->m2 = 0;
  for (int32_t v = 0; v < n; v++) {
    if (col[v] != c) continue;
    if (w[v] > s->m1) {
      s->m2 = s->m1;
      s->m1 = w[v];
      s->cnt1 = 1;
    } else if (w[v] == s->m1) {
      s->cnt1++;
    } else if (w[v] > s->m2) {
      s->m2 = w[v];
    }
  }
}

/*
 * Algorithm 2 for one individual.  Round r runs `iters_per_round` tabu
 * iterations minimising g = (f_w << shift) + phi * c, where phi is a
 * fixed-point penalty (shift fractional bits): phi_0 = k * max_w / (2 n),
 * halved after a round whose best state is legal, doubled otherwise, and
 * 2 * max_w in the last round.  The moved vertex is frozen for
 * L + floor(frz_num * n / frz_den) iterations.  Every round starts from the
 * best-g state of the previous one; the best legal colouring met anywhere is
 * the result.  colors: in = start, out = best legal (or the last round's
 * best-g state if no legal colouring was met).  best_legal = INT32_MAX when
 * none.  stats: 0 moves, 1 no-ops, 2 sum deg(v*), 3 tie iterations,
 * 4 rounds ending legal, 5 final phi (fixed point).
 * trace (optional, trace_cap records over all rounds): {v | c << 16, g after
 * the move}; a no-op records v = c = 0xffff.  round_log (optional,
 * [rounds][3]): phi used in the round, 1 if the round's best-g state is
 * legal, f_w of that state.
 */
int orc_wvcp_tabu(int32_t n, const int32_t* rp, const int32_t* ci, const int32_t* w,
                  const orc_wvcp_params* p, int32_t ind, int16_t* colors, int32_t* best_legal_out,
                  int64_t* stats, uint64_t* hash_out, int64_t* trace, int32_t trace_cap,
                  int64_t* round_log) {
  const int32_t k = p->k;
  const int S = p->shift;
  int16_t* col = (int16_t*)malloc(sizeof(int16_t) * (size_t)n);
  int16_t* bestg = (int16_t*)malloc(sizeof(int16_t) * (size_t)n);
  int16_t* bestl = (int16_t*)malloc(sizeof(int16_t) * (size_t)n);
  int32_t* gamma = (int32_t*)calloc((size_t)n * k, sizeof(int32_t));
  int64_t* frozen = (int64_t*)calloc((size_t)n, sizeof(int64_t));
  cls_t* cs = (cls_t*)calloc((size_t)k, sizeof(cls_t));
  int rc = 0;
  for (int s = 0; s < ORC_NSTATS; s++) stats[s] = 0;
  memcpy(col, colors, sizeof(int16_t) * (size_t)n);
  int64_t maxw = 0;
  for (int32_t v = 0; v < n; v++)
    if (w[v] > maxw) maxw = w[v];
  int64_t phi = ((int64_t)k * maxw << S) / (2 * (int64_t)n);
  const int64_t PHI_MAX = (int64_t)1 << 30;
  int64_t best_legal = INT64_MAX;
  int have_legal = 0;
  uint64_t h = FNV_OFF;
  int64_t t = 0;
  const uint32_t uind = (uint32_t)ind;
  const int64_t frz = (int64_t)p->frz_num * n / p->frz_den;

  for (int32_t r = 0; r < p->rounds; r++) {
    if (r == p->rounds - 1) phi = (2 * maxw) << S;
    /* fresh search state for this round */
    memset(gamma, 0, sizeof(int32_t) * (size_t)n * k);
    for (int32_t v = 0; v < n; v++)
      for (int32_t e = rp[v]; e < rp[v + 1]; e++) gamma[(int64_t)v * k + col[ci[e]]]++;
    for (int32_t v = 0; v < n; v++) frozen[v] = 0;
    for (int32_t c = 0; c < k; c++) class_stats(n, w, col, c, &cs[c]);
    int64_t conf = orc_conflicts(n, rp, ci, col);
    int64_t fw = orc_wscore(n, w, k, col);
    int64_t g = (fw << S) + phi * conf;
    int64_t g_best = g;
    memcpy(bestg, col, sizeof(int16_t) * (size_t)n);
    if (conf == 0 && fw < best_legal) {
      best_legal = fw;
      have_legal = 1;
      memcpy(bestl, col, sizeof(int16_t) * (size_t)n);
    }
    for (int64_t it = 0; it < p->iters_per_round; it++, t++) {
      cand_t bestc;
      bestc.v = -1;
      bestc.has_h = 0;
      int64_t nmin = 0;
      for (int32_t v = 0; v < n; v++) {
        int32_t a = col[v];
        int64_t wv = w[v];
        /* largest weight left in class a once v leaves it */
        int64_t m_after = (wv < cs[a].m1 || cs[a].cnt1 > 1) ? cs[a].m1 : cs[a].m2;
        int64_t d_leave = m_after - cs[a].m1;
        int32_t gcur = gamma[(int64_t)v * k + a];
        for (int32_t c = 0; c < k; c++) {
          if (c == a) continue;
          int64_t d_join = (wv > cs[c].m1 ? wv : cs[c].m1) - cs[c].m1;
          int64_t dfw = d_join + d_leave;
          int64_t dc = (int64_t)gamma[(int64_t)v * k + c] - gcur;
          int64_t dg = (dfw << S) + phi * dc;
          if (frozen[v] > t && !(g + dg < g_best)) continue;
          cand_t cc = {dg, 0, 0, v, c};
          if (bestc.v >= 0 && dg == bestc.d) nmin++;
          else if (bestc.v < 0 || dg < bestc.d) nmin = 1;
          if (cand_better(&cc, &bestc, p->seed, uind, (uint32_t)t)) bestc = cc;
        }
      }
      if (nmin >= 2) stats[3]++;
      if (bestc.v < 0) {
        stats[1]++;
        h = fnv_step(h, 0xffffu, 0xffffu, g >> S);
        if (trace && t < trace_cap) {
          trace[2 * t] = 0xffffffffll;
          trace[2 * t + 1] = g;
        }
        continue;
      }
      const int32_t v = bestc.v, c = bestc.c, a = col[v];
      col[v] = (int16_t)c;
      int64_t dc = (int64_t)gamma[(int64_t)v * k + c] - gamma[(int64_t)v * k + a];
      for (int32_t e = rp[v]; e < rp[v + 1]; e++) {
        int32_t u = ci[e];
        gamma[(int64_t)u * k + a]--;
        gamma[(int64_t)u * k + c]++;
      }
      class_stats(n, w, col, a, &cs[a]);
      class_stats(n, w, col, c, &cs[c]);
      conf += dc;
      g += bestc.d;
      fw = (g - phi * conf) >> S;
      if (p->check) {
        int64_t fw2 = orc_wscore(n, w, k, col), conf2 = orc_conflicts(n, rp, ci, col);
        if (fw2 != fw || conf2 != conf || (fw2 << S) + phi * conf2 != g) {
          snprintf(orc_err, sizeof orc_err,
                   "wvcp ind %d t %lld: fw %lld/%lld conf %lld/%lld", ind, (long long)t,
                   (long long)fw, (long long)fw2, (long long)conf, (long long)conf2);
          rc = -1;
          goto done;
        }
      }
      int64_t L = orc_uniform(word0(uind, (uint32_t)t, 0, D_TENURE, p->seed), (uint32_t)p->ten_rand);
      frozen[v] = t + L + frz;
      if (g < g_best) {
        g_best = g;
        memcpy(bestg, col, sizeof(int16_t) * (size_t)n);
      }
      if (conf == 0 && fw < best_legal) {
        best_legal = fw;
        have_legal = 1;
        memcpy(bestl, col, sizeof(int16_t) * (size_t)n);
      }
      stats[0]++;
      stats[2] += rp[v + 1] - rp[v];
      h = fnv_step(h, (uint32_t)v, (uint32_t)c, g >> S);
      if (trace && t < trace_cap) {
        trace[2 * t] = (int64_t)((v & 0xffff) | (c << 16));
        trace[2 * t + 1] = g;
      }
    }
    /* next round starts from this round's best-g state */
    memcpy(col, bestg, sizeof(int16_t) * (size_t)n);
    int legal = orc_conflicts(n, rp, ci, col) == 0;
    stats[4] += legal;
    if (round_log) {
      round_log[3 * r] = phi;
      round_log[3 * r + 1] = legal;
      round_log[3 * r + 2] = orc_wscore(n, w, k, col);
    }
    if (r < p->rounds - 1) {
      if (legal) phi >>= 1;
      else phi = (phi << 1) > PHI_MAX ? PHI_MAX : (phi << 1);
    }
  }
  stats[5] = phi;
done:
  if (have_legal) memcpy(colors, bestl, sizeof(int16_t) * (size_t)n);
  else memcpy(colors, col, sizeof(int16_t) * (size_t)n);
  *best_legal_out = have_legal ? (int32_t)best_legal : INT32_MAX;
  *hash_out = h;
  free(col);
  free(bestg);
  free(bestl);
  free(gamma);
  free(frozen);
  free(cs);
  return rc;
}

int orc_wvcp_batch(int32_t n, const int32_t* rp, const int32_t* ci, const int32_t* w,
                   const orc_wvcp_params* p, int32_t count, const int32_t* ind_ids,
                   int16_t* colors, int32_t* best_legal, int64_t* stats, uint64_t* hashes,
                   int32_t nthreads) {
  int rc = 0;
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads) reduction(| : rc)
  for (int32_t i = 0; i < count; i++) {
    int r = orc_wvcp_tabu(n, rp, ci, w, p, ind_ids[i], colors + (int64_t)i * n, best_legal + i,
                          stats + (int64_t)i * ORC_NSTATS, hashes + i, NULL, 0, NULL);
    rc |= (r != 0);
  }
  return rc ? -1 : 0;
}

/* ------------------------------------------------------------------ */
/* Greedy partition crossover (GPX).                                   */
/* ------------------------------------------------------------------ */
/*
 * Step l = 0..k-1 takes parent A when l is even, B when l is odd, picks the
 * class of that parent with the most still-unassigned vertices (ties: the
 * smaller Philox word of (child, l, lowest unassigned vertex of the class),
 * then that vertex), and gives its unassigned vertices colour l.  Vertices
 * still unassigned after k steps get a uniform random colour.
 */
void orc_gpx(int32_t n, int32_t k, const int16_t* A, const int16_t* B, uint32_t child,
             uint64_t seed, int16_t* out) {
  unsigned char* done = (unsigned char*)calloc((size_t)n, 1);
  int32_t* size = (int32_t*)malloc(sizeof(int32_t) * (size_t)k);
  int32_t* minv = (int32_t*)malloc(sizeof(int32_t) * (size_t)k);
  for (int32_t l = 0; l < k; l++) {
    const int16_t* P = (l % 2 == 0) ? A : B;
    for (int32_t c = 0; c < k; c++) {
      size[c] = 0;
      minv[c] = n;
    }
    for (int32_t v = 0; v < n; v++) {
      if (done[v]) continue;
      size[P[v]]++;
      if (v < minv[P[v]]) minv[P[v]] = v;
    }
    int32_t bc = -1;
    uint32_t bh = 0;
    for (int32_t c = 0; c < k; c++) {
      if (size[c] == 0) continue;
      if (bc < 0 || size[c] > size[bc]) {
        bc = c;
        bh = word0(child, (uint32_t)l, (uint32_t)minv[c], D_GPXTIE, seed);
      } else if (size[c] == size[bc]) {
        uint32_t hc = word0(child, (uint32_t)l, (uint32_t)minv[c], D_GPXTIE, seed);
        if (hc < bh || (hc == bh && minv[c] < minv[bc])) {
          bc = c;
          bh = hc;
        }
      }
    }
    if (bc < 0) break; /* everything assigned */
    for (int32_t v = 0; v < n; v++)
      if (!done[v] && P[v] == bc) {
        out[v] = (int16_t)l;
        done[v] = 1;
      }
  }
  for (int32_t v = 0; v < n; v++)
    if (!done[v])
      out[v] = (int16_t)orc_uniform(word0(child, 0, (uint32_t)v, D_GPXFILL, seed), (uint32_t)k);
  free(done);
  free(size);
  free(minv);
}

/* children[(p*per_pair + j)] = GPX(parents[pairs[p][0]], parents[pairs[p][1]]), child id
 * child_base + p*per_pair + j */
void orc_gpx_batch(int32_t n, int32_t k, const int16_t* parents, const int32_t* pairs,
                   int32_t npairs, int32_t per_pair, uint32_t child_base, uint64_t seed,
                   int16_t* children) {
  for (int32_t p = 0; p < npairs; p++)
    for (int32_t j = 0; j < per_pair; j++) {
      int64_t ci = (int64_t)p * per_pair + j;
      orc_gpx(n, k, parents + (int64_t)pairs[2 * p] * n, parents + (int64_t)pairs[2 * p + 1] * n,
              child_base + (uint32_t)ci, seed, children + ci * n);
    }
}

/* ------------------------------------------------------------------ */
/* Offspring selection (eq. select_cross, population-wide reading).     */
/* ------------------------------------------------------------------ */
/* total order on floats: -inf < ... < +inf < NaN */
static uint32_t float_key(float x) {
  uint32_t u;
  memcpy(&u, &x, 4);
  if (x != x) return 0xffffffffu;
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

/*
 * mode 0 (learned): the `keep` offspring with the smallest predicted score,
 * ties by index.  mode 1 (plain): the `keep` offspring with the smallest
 * Philox word of (i, gen, 0, D_SELECT), ties by index.  idx_out lists them
 * in that order.  Plain O(count^2) ranking.
 */
void orc_select(const float* scores, int32_t count, int32_t keep, int32_t mode, uint64_t seed,
                uint32_t gen, int32_t* idx_out) {
  uint32_t* key = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(count > 0 ? count : 1));
  for (int32_t i = 0; i < count; i++)
    key[i] = mode == 0 ? float_key(scores[i]) : word0((uint32_t)i, gen, 0, D_SELECT, seed);
  for (int32_t i = 0; i < count; i++) {
    int32_t rank = 0;
    for (int32_t j = 0; j < count; j++)
      if (key[j] < key[i] || (key[j] == key[i] && j < i)) rank++;
    if (rank < keep) idx_out[rank] = i;
  }
  free(key);
}

/* ------------------------------------------------------------------ */
/* Parent pairing of the simplified generation: individual i crosses   */
/* with a uniform other member j (Philox counter (i, gen, 0, 0x80000009)). */
/* ------------------------------------------------------------------ */
void orc_random_pairs(int32_t pop, uint64_t seed, uint32_t gen, int32_t* pairs) {
  for (int32_t i = 0; i < pop; i++) {
    int32_t j = 0;
    if (pop > 1) {
      j = (int32_t)orc_uniform(word0((uint32_t)i, gen, 0, 0x80000009u, seed), (uint32_t)(pop - 1));
      if (j >= i) j++;
    }
    pairs[2 * i] = i;
    pairs[2 * i + 1] = j;
  }
}
