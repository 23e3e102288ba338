/*
 * FP64 CPU oracle for exhaustive, constrained top-k retrieval over a
 * combinatorial synthesis library (CSL) scored by a factorised surrogate.
 *
 * TEST INFRASTRUCTURE ONLY. It is loaded by the tests, by the smoke check and by
 * the CPU-baseline leg of the benchmark, never by the product path, and it
 * shares no code with the HIP library.
 *
 * What it computes, in the paper's terms:
 *   - A library D = (T, R, S, psi, phi): reactions t, each with 2 or 3 R-groups
 *     ("slots"), each slot with a set of synthons (Section 4.2; Appendix A.1).
 *     A compound is the multi-index chi = (t, {(r, s)}) with one synthon per slot.
 *   - Its embedding is the sum of the per-(R-group, synthon) associative
 *     embeddings u_{r,s} (eq. "factorizer"), here given directly as table rows.
 *   - The heads are a decoder applied to that sum. With one layer this is the
 *     paper's linear probe f_i = w_i^T g + b_i (eq. "surrogate"), and the result
 *     equals the APEX factorisation sum_{(r,s)} v_{i,r,s} + b_i (eq. "apex").
 *     Deeper decoders (Linear -> act -> ... -> Linear) generalise it.
 *   - The query maximises sum of the objective over at most k compounds subject
 *     to l_i <= f_i <= u_i for every selected compound (eq. "apex_topk"). Its
 *     solution is the k best feasible compounds; equal objectives are ordered by
 *     lower compound id. The objective here is a weighted sum w . heads, which
 *     covers a single head, a negated head and the composite objectives of
 *     Appendix A.11.
 *   - orc_topk_lex keeps the paper's own formulation: a size-k priority queue
 *     ordered lexicographically by (violation c, objective), where
 *     c = -sum max(0, l_i - f_i) - sum max(0, f_i - u_i), followed by removal of
 *     entries with c < 0 (Section 4.3, violation equation). Skipping that
 *     removal gives the violation-ranked fallback: when fewer than k compounds
 *     are feasible, the least-violating ones fill the remaining places.
 *   - Values the paper does not cover: a compound whose objective or any head
 *     is NaN or +-Inf is never a candidate (in either form).
 *
 * Everything is evaluated in double precision from the float32 inputs, by
 * plain loops: the sum of table rows in slot order, then each layer as
 * out_j = b_j + sum_i W_ji x_i, then the activation, then a full sort.
 *
 * Compound ids (reading of the paper's multi-index as one integer): reactions in
 * order, and inside reaction t the assignment (i0, i1[, i2]) in row-major order
 * with slot 0 most significant:
 *   id = offset_t + (i0 * n1 + i1) * n2 + i2    (n2 = 1, i2 = 0 for two slots).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_ACT_NONE 0
#define ORC_ACT_RELU 1
#define ORC_ACT_SILU 2

typedef struct {
  uint32_t n_reactions;
  const uint32_t* n_slots;    /* [T] */
  const uint32_t* slot_sizes; /* [sum n_slots] */
  uint32_t d;
  const float* tables; /* [rows x d], rows in (reaction, slot, synthon) order */
} orc_library;

typedef struct {
  uint32_t n_layers;
  const uint32_t* dims; /* [n_layers + 1] */
  uint32_t act;
  const float* const* W; /* W[l]: dims[l+1] x dims[l], row-major */
  const float* const* b; /* b[l]: dims[l+1] */
} orc_decoder;

typedef struct {
  const float* w; /* objective weights [H] */
  uint32_t n_con;
  const uint32_t* con_head;
  const float* con_lo; /* inclusive, may be -inf */
  const float* con_hi; /* inclusive, may be +inf */
  uint64_t k;
  const uint8_t* subset; /* [T] 1 = reaction searched; NULL = all */
} orc_query;

typedef struct {
  uint64_t id;
  double o;
} orc_entry;

/* ------------------------------------------------------------------------ */
/* Library bookkeeping: counts and the multi-index <-> id map.              */
/* ------------------------------------------------------------------------ */

static uint64_t reaction_count(const orc_library* L, uint32_t t, const uint32_t* slot_base) {
  uint64_t c = 1;
  for (uint32_t s = 0; s < L->n_slots[t]; s++) c *= (uint64_t)L->slot_sizes[slot_base[t] + s];
  return c;
}

/* slot_base[t] = index of reaction t's first slot; row_base[j] = first table row
 * of slot j; offset[t] = id of the first compound of reaction t. */
static void layout(const orc_library* L, uint32_t* slot_base, uint64_t* row_base, uint64_t* offset) {
  uint32_t sb = 0;
  uint64_t rb = 0, off = 0;
  for (uint32_t t = 0; t < L->n_reactions; t++) {
    slot_base[t] = sb;
    for (uint32_t s = 0; s < L->n_slots[t]; s++) {
      row_base[sb + s] = rb;
      rb += L->slot_sizes[sb + s];
    }
    offset[t] = off;
    off += reaction_count(L, t, slot_base);
    sb += L->n_slots[t];
  }
  offset[L->n_reactions] = off;
}

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

uint64_t orc_num_compounds(const orc_library* L) {
  uint64_t total = 0;
  uint32_t sb = 0;
  for (uint32_t t = 0; t < L->n_reactions; t++) {
    uint64_t c = 1;
    for (uint32_t s = 0; s < L->n_slots[t]; s++) c *= (uint64_t)L->slot_sizes[sb + s];
    total += c;
    sb += L->n_slots[t];
  }
  return total;
}

/* id -> (reaction, synthon index per slot); unused third slot gets 0. Returns 0
 * on success, -1 if the id is out of range. */
int orc_decode(const orc_library* L, const uint64_t* ids, uint64_t n, uint32_t* reaction,
               uint32_t* synthon /* [n x 3] */) {
  uint32_t* slot_base = (uint32_t*)malloc(sizeof(uint32_t) * (L->n_reactions + 1));
  uint64_t* row_base = (uint64_t*)malloc(sizeof(uint64_t) * 3 * (L->n_reactions + 1));
  uint64_t* offset = (uint64_t*)malloc(sizeof(uint64_t) * (L->n_reactions + 1));
  layout(L, slot_base, row_base, offset);
  int rc = 0;
  for (uint64_t q = 0; q < n; q++) {
    uint64_t id = ids[q];
    if (id >= offset[L->n_reactions]) {
      rc = -1;
      break;
    }
    uint32_t t = 0;
    while (offset[t + 1] <= id) t++; /* linear scan: plain, not fast */
    uint64_t r = id - offset[t];
    uint32_t ns = L->n_slots[t];
    uint32_t idx[3] = {0, 0, 0};
    for (int s = (int)ns - 1; s >= 0; s--) {
      uint64_t n_s = L->slot_sizes[slot_base[t] + (uint32_t)s];
      idx[s] = (uint32_t)(r % n_s);
      r /= n_s;
    }
    reaction[q] = t;
    synthon[3 * q + 0] = idx[0];
    synthon[3 * q + 1] = idx[1];
    synthon[3 * q + 2] = idx[2];
  }
  free(slot_base);
  free(row_base);
  free(offset);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* The surrogate on one compound.                                           */
/* ------------------------------------------------------------------------ */

typedef struct {
  uint32_t n_layers, act, H, maxw;
  const uint32_t* dims;
  double** W; /* promoted copies */
  double** b;
} dec64;

static void dec64_init(dec64* D, const orc_decoder* dec) {
  D->n_layers = dec->n_layers;
  D->act = dec->act;
  D->dims = dec->dims;
  D->H = dec->dims[dec->n_layers];
  D->maxw = 0;
  for (uint32_t l = 0; l <= dec->n_layers; l++)
    if (dec->dims[l] > D->maxw) D->maxw = dec->dims[l];
  D->W = (double**)malloc(sizeof(double*) * dec->n_layers);
  D->b = (double**)malloc(sizeof(double*) * dec->n_layers);
  for (uint32_t l = 0; l < dec->n_layers; l++) {
    size_t nw = (size_t)dec->dims[l + 1] * dec->dims[l];
    D->W[l] = (double*)malloc(sizeof(double) * nw);
    D->b[l] = (double*)malloc(sizeof(double) * dec->dims[l + 1]);
    for (size_t i = 0; i < nw; i++) D->W[l][i] = (double)dec->W[l][i];
    for (uint32_t j = 0; j < dec->dims[l + 1]; j++) D->b[l][j] = (double)dec->b[l][j];
  }
}

static void dec64_free(dec64* D) {
  for (uint32_t l = 0; l < D->n_layers; l++) {
    free(D->W[l]);
    free(D->b[l]);
  }
  free(D->W);
  free(D->b);
}

static double activation(uint32_t act, double v) {
  if (act == ORC_ACT_RELU) return v > 0.0 ? v : 0.0;
  if (act == ORC_ACT_SILU) return v / (1.0 + exp(-v));
  return v;
}

/* heads = decoder(sum of the compound's table rows). x, y: scratch of maxw. */
static void forward_compound(const orc_library* L, const dec64* D, const uint64_t* rows, uint32_t nrows,
                             double* x, double* y, double* heads) {
  const uint32_t d = L->d;
  /* eq. "factorizer": g = sum over the compound's (R-group, synthon) pairs of u_{r,s} */
  for (uint32_t c = 0; c < d; c++) x[c] = 0.0;
  for (uint32_t s = 0; s < nrows; s++) {
    const float* u = L->tables + rows[s] * (uint64_t)d;
    for (uint32_t c = 0; c < d; c++) x[c] += (double)u[c];
  }
  /* decoder layers: out_j = b_j + sum_i W_ji in_i, activation between layers */
  double* in = x;
  double* out = y;
  for (uint32_t l = 0; l < D->n_layers; l++) {
    const uint32_t ni = D->dims[l], no = D->dims[l + 1];
    const double* W = D->W[l];
    for (uint32_t j = 0; j < no; j++) {
      double acc = D->b[l][j];
      for (uint32_t i = 0; i < ni; i++) acc += W[(size_t)j * ni + i] * in[i];
      out[j] = (l + 1 < D->n_layers) ? activation(D->act, acc) : acc;
    }
    double* tmp = in;
    in = out;
    out = tmp;
  }
  for (uint32_t h = 0; h < D->H; h++) heads[h] = in[h];
}

/* Objective and feasibility (Section 4 problem statement, bounds inclusive). */
static double objective(const orc_query* Q, const double* heads, uint32_t H) {
  double o = 0.0;
  for (uint32_t h = 0; h < H; h++) o += (double)Q->w[h] * heads[h];
  return o;
}

/* Reading of the problem statement for values it does not cover: a compound
 * whose objective or any head is not a finite number (NaN or +-Inf) has no
 * meaningful score and is never a candidate, whatever its bounds. */
static int finite_compound(double o, const double* heads, uint32_t H) {
  if (!isfinite(o)) return 0;
  for (uint32_t h = 0; h < H; h++)
    if (!isfinite(heads[h])) return 0;
  return 1;
}

static int feasible(const orc_query* Q, const double* heads) {
  for (uint32_t c = 0; c < Q->n_con; c++) {
    double f = heads[Q->con_head[c]];
    if (!(f >= (double)Q->con_lo[c] && f <= (double)Q->con_hi[c])) return 0;
  }
  return 1;
}

/* The violation of the violation equation (Section 4.3): zero iff feasible. */
static double violation(const orc_query* Q, const double* heads) {
  double c = 0.0;
  for (uint32_t i = 0; i < Q->n_con; i++) {
    double f = heads[Q->con_head[i]];
    double lo = (double)Q->con_lo[i], hi = (double)Q->con_hi[i];
    c -= (lo - f > 0.0) ? (lo - f) : 0.0;
    c -= (f - hi > 0.0) ? (f - hi) : 0.0;
  }
  return c;
}

/* Distance from the nearest bound, positive when inside all bounds. */
static double slack(const orc_query* Q, const double* heads) {
  double m = INFINITY;
  for (uint32_t i = 0; i < Q->n_con; i++) {
    double f = heads[Q->con_head[i]];
    double a = f - (double)Q->con_lo[i];
    double b = (double)Q->con_hi[i] - f;
    double s = a < b ? a : b;
    if (s < m) m = s;
  }
  return m;
}

static int cmp_entry(const void* pa, const void* pb) {
  const orc_entry* a = (const orc_entry*)pa;
  const orc_entry* b = (const orc_entry*)pb;
  if (a->o > b->o) return -1;
  if (a->o < b->o) return 1;
  if (a->id < b->id) return -1;
  if (a->id > b->id) return 1;
  return 0;
}

/* Pointwise heads for a list of ids: heads[n x H]. */
int orc_heads(const orc_library* L, const orc_decoder* dec, const uint64_t* ids, uint64_t n,
              double* heads_out) {
  uint32_t* reaction = (uint32_t*)malloc(sizeof(uint32_t) * (n ? n : 1));
  uint32_t* syn = (uint32_t*)malloc(sizeof(uint32_t) * 3 * (n ? n : 1));
  if (orc_decode(L, ids, n, reaction, syn) != 0) {
    free(reaction);
    free(syn);
    return -1;
  }
  uint32_t* slot_base = (uint32_t*)malloc(sizeof(uint32_t) * (L->n_reactions + 1));
  uint64_t* row_base = (uint64_t*)malloc(sizeof(uint64_t) * 3 * (L->n_reactions + 1));
  uint64_t* offset = (uint64_t*)malloc(sizeof(uint64_t) * (L->n_reactions + 1));
  layout(L, slot_base, row_base, offset);
  dec64 D;
  dec64_init(&D, dec);
#pragma omp parallel
  {
    double* x = (double*)malloc(sizeof(double) * (D.maxw > L->d ? D.maxw : L->d));
    double* y = (double*)malloc(sizeof(double) * (D.maxw > L->d ? D.maxw : L->d));
#pragma omp for schedule(dynamic, 64)
    for (int64_t q = 0; q < (int64_t)n; q++) {
      uint32_t t = reaction[q];
      uint64_t rows[3];
      for (uint32_t s = 0; s < L->n_slots[t]; s++)
        rows[s] = row_base[slot_base[t] + s] + syn[3 * q + s];
      forward_compound(L, &D, rows, L->n_slots[t], x, y, heads_out + (uint64_t)q * D.H);
    }
    free(x);
    free(y);
  }
  dec64_free(&D);
  free(slot_base);
  free(row_base);
  free(offset);
  free(reaction);
  free(syn);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Exhaustive top-k (eq. "apex_topk"): enumerate everything, keep feasible   */
/* compounds, full sort by (objective desc, id asc), take the first k.       */
/* ------------------------------------------------------------------------ */

typedef struct {
  orc_entry* v;
  uint64_t n, cap;
} vec_t;

static void vec_push(vec_t* a, uint64_t id, double o) {
  if (a->n == a->cap) {
    a->cap = a->cap ? a->cap * 2 : 1024;
    a->v = (orc_entry*)realloc(a->v, sizeof(orc_entry) * a->cap);
  }
  a->v[a->n].id = id;
  a->v[a->n].o = o;
  a->n++;
}

typedef struct {
  uint64_t n_feasible;
  uint64_t n_out;
  double min_slack_selected;  /* over returned top-k entries; +inf if no constraint */
  double min_violation_near;  /* over infeasible compounds with o >= o_(k+1); +inf if none */
  uint64_t n_near;            /* infeasible compounds within near_tol of feasibility */
} orc_topk_info;

/* out_* hold min(k + extra, n_feasible) entries. near_tol: infeasible compounds
 * whose worst bound violation is <= near_tol are tracked for the margin report. */
int orc_topk(const orc_library* L, const orc_decoder* dec, const orc_query* Q, int nthreads,
             uint64_t extra, double near_tol, uint64_t* out_ids, double* out_o, double* out_heads,
             orc_topk_info* info) {
  const uint32_t T = L->n_reactions;
  if (dec->dims[0] != L->d) return -1;
  for (uint32_t c = 0; c < Q->n_con; c++)
    if (Q->con_head[c] >= dec->dims[dec->n_layers]) return -1;
  uint32_t* slot_base = (uint32_t*)malloc(sizeof(uint32_t) * (T + 1));
  uint64_t* row_base = (uint64_t*)malloc(sizeof(uint64_t) * 3 * (T + 1));
  uint64_t* offset = (uint64_t*)malloc(sizeof(uint64_t) * (T + 1));
  layout(L, slot_base, row_base, offset);
  dec64 D;
  dec64_init(&D, dec);
  const uint32_t H = D.H;

  /* work items: (reaction, synthon of slot 0) */
  uint64_t n_items = 0;
  for (uint32_t t = 0; t < T; t++) n_items += L->slot_sizes[slot_base[t]];
  uint32_t* item_t = (uint32_t*)malloc(sizeof(uint32_t) * (n_items ? n_items : 1));
  uint32_t* item_i = (uint32_t*)malloc(sizeof(uint32_t) * (n_items ? n_items : 1));
  {
    uint64_t p = 0;
    for (uint32_t t = 0; t < T; t++)
      for (uint32_t i = 0; i < L->slot_sizes[slot_base[t]]; i++) {
        item_t[p] = t;
        item_i[p] = i;
        p++;
      }
  }

#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
  int nt = omp_get_max_threads();
#else
  int nt = 1;
#endif
  vec_t* feas = (vec_t*)calloc((size_t)nt, sizeof(vec_t));
  vec_t* near = (vec_t*)calloc((size_t)nt, sizeof(vec_t)); /* o stored, violation in id slot */
  double** nearv = (double**)calloc((size_t)nt, sizeof(double*));
  uint64_t* nearcap = (uint64_t*)calloc((size_t)nt, sizeof(uint64_t));

#pragma omp parallel
  {
#ifdef _OPENMP
    int tid = omp_get_thread_num();
#else
    int tid = 0;
#endif
    uint32_t w = D.maxw > L->d ? D.maxw : L->d;
    double* x = (double*)malloc(sizeof(double) * w);
    double* y = (double*)malloc(sizeof(double) * w);
    double* heads = (double*)malloc(sizeof(double) * H);
#pragma omp for schedule(dynamic, 1)
    for (int64_t it = 0; it < (int64_t)n_items; it++) {
      uint32_t t = item_t[it], i0 = item_i[it];
      if (Q->subset && !Q->subset[t]) continue;
      uint32_t ns = L->n_slots[t];
      uint32_t n1 = L->slot_sizes[slot_base[t] + 1];
      uint32_t n2 = ns == 3 ? L->slot_sizes[slot_base[t] + 2] : 1;
      for (uint32_t i1 = 0; i1 < n1; i1++)
        for (uint32_t i2 = 0; i2 < n2; i2++) {
          uint64_t rows[3];
          rows[0] = row_base[slot_base[t] + 0] + i0;
          rows[1] = row_base[slot_base[t] + 1] + i1;
          rows[2] = ns == 3 ? row_base[slot_base[t] + 2] + i2 : 0;
          uint64_t id = offset[t] + ((uint64_t)i0 * n1 + i1) * n2 + i2;
          forward_compound(L, &D, rows, ns, x, y, heads);
          double o = objective(Q, heads, H);
          if (!finite_compound(o, heads, H)) continue;
          if (feasible(Q, heads)) {
            vec_push(&feas[tid], id, o);
          } else if (-violation(Q, heads) <= near_tol * (double)(Q->n_con ? Q->n_con : 1)) {
            double worst = 0.0;
            for (uint32_t c = 0; c < Q->n_con; c++) {
              double f = heads[Q->con_head[c]];
              double v1 = (double)Q->con_lo[c] - f, v2 = f - (double)Q->con_hi[c];
              double v = v1 > v2 ? v1 : v2;
              if (v > worst) worst = v;
            }
            if (worst <= near_tol) {
              vec_push(&near[tid], id, o);
              if (near[tid].n > nearcap[tid]) {
                nearcap[tid] = near[tid].cap;
                nearv[tid] = (double*)realloc(nearv[tid], sizeof(double) * nearcap[tid]);
              }
              nearv[tid][near[tid].n - 1] = worst;
            }
          }
        }
    }
    free(x);
    free(y);
    free(heads);
  }

  uint64_t nf = 0;
  for (int t = 0; t < nt; t++) nf += feas[t].n;
  orc_entry* all = (orc_entry*)malloc(sizeof(orc_entry) * (nf ? nf : 1));
  {
    uint64_t p = 0;
    for (int t = 0; t < nt; t++) {
      if (feas[t].n) memcpy(all + p, feas[t].v, sizeof(orc_entry) * feas[t].n);
      p += feas[t].n;
      free(feas[t].v);
    }
  }
  qsort(all, nf, sizeof(orc_entry), cmp_entry);
  uint64_t n_out = Q->k + extra < nf ? Q->k + extra : nf;
  for (uint64_t q = 0; q < n_out; q++) {
    out_ids[q] = all[q].id;
    out_o[q] = all[q].o;
  }
  if (out_heads && n_out) orc_heads(L, dec, out_ids, n_out, out_heads);

  info->n_feasible = nf;
  info->n_out = n_out;
  /* margins: how far the returned set is from changing under small errors */
  info->min_slack_selected = INFINITY;
  if (out_heads) {
    uint64_t kk = Q->k < n_out ? Q->k : n_out;
    for (uint64_t q = 0; q < kk; q++) {
      double s = slack(Q, out_heads + q * H);
      if (s < info->min_slack_selected) info->min_slack_selected = s;
    }
  }
  double cut = nf > Q->k ? all[Q->k].o : -INFINITY; /* o_(k+1) */
  info->min_violation_near = INFINITY;
  info->n_near = 0;
  for (int t = 0; t < nt; t++) {
    for (uint64_t q = 0; q < near[t].n; q++) {
      info->n_near++;
      if (near[t].v[q].o >= cut && nearv[t][q] < info->min_violation_near)
        info->min_violation_near = nearv[t][q];
    }
    free(near[t].v);
    free(nearv[t]);
  }
  free(near);
  free(nearv);
  free(nearcap);
  free(feas);
  free(all);
  free(item_t);
  free(item_i);
  dec64_free(&D);
  free(slot_base);
  free(row_base);
  free(offset);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* The paper's literal form (Section 4.3): a size-k priority queue over       */
/* (violation, objective) in lexicographic order, ties by lower id, then drop */
/* entries with negative violation. Single-threaded, for small libraries.     */
/* Without the final removal the same queue is the violation-ranked fallback. */
/* ------------------------------------------------------------------------ */

typedef struct {
  double c, o;
  uint64_t id;
} lex_entry;

/* 1 if a ranks before (is better than) b */
static int lex_better(const lex_entry* a, const lex_entry* b) {
  if (a->c != b->c) return a->c > b->c;
  if (a->o != b->o) return a->o > b->o;
  return a->id < b->id;
}

/* keep_violators = 0: the paper's result (violators removed at the end).
 * keep_violators = 1: the queue as it stands after the last compound, so that
 * when fewer than k compounds are feasible the remaining places go to the
 * least-violating compounds (best violation first, then objective, then id);
 * out_c receives each entry's violation (<= 0) when it is not NULL. */
int orc_topk_lex(const orc_library* L, const orc_decoder* dec, const orc_query* Q, int keep_violators,
                 uint64_t* out_ids, double* out_o, double* out_c, uint64_t* n_out) {
  const uint32_t T = L->n_reactions;
  uint32_t* slot_base = (uint32_t*)malloc(sizeof(uint32_t) * (T + 1));
  uint64_t* row_base = (uint64_t*)malloc(sizeof(uint64_t) * 3 * (T + 1));
  uint64_t* offset = (uint64_t*)malloc(sizeof(uint64_t) * (T + 1));
  layout(L, slot_base, row_base, offset);
  dec64 D;
  dec64_init(&D, dec);
  uint32_t w = D.maxw > L->d ? D.maxw : L->d;
  double* x = (double*)malloc(sizeof(double) * w);
  double* y = (double*)malloc(sizeof(double) * w);
  double* heads = (double*)malloc(sizeof(double) * D.H);
  /* the queue: a sorted array, best first; insertion by shifting */
  lex_entry* qv = (lex_entry*)malloc(sizeof(lex_entry) * (Q->k + 1));
  uint64_t qn = 0;
  for (uint32_t t = 0; t < T; t++) {
    if (Q->subset && !Q->subset[t]) continue;
    uint32_t ns = L->n_slots[t];
    uint32_t n0 = L->slot_sizes[slot_base[t]];
    uint32_t n1 = L->slot_sizes[slot_base[t] + 1];
    uint32_t n2 = ns == 3 ? L->slot_sizes[slot_base[t] + 2] : 1;
    for (uint32_t i0 = 0; i0 < n0; i0++)
      for (uint32_t i1 = 0; i1 < n1; i1++)
        for (uint32_t i2 = 0; i2 < n2; i2++) {
          uint64_t rows[3] = {row_base[slot_base[t]] + i0, row_base[slot_base[t] + 1] + i1,
                              ns == 3 ? row_base[slot_base[t] + 2] + i2 : 0};
          lex_entry e;
          e.id = offset[t] + ((uint64_t)i0 * n1 + i1) * n2 + i2;
          forward_compound(L, &D, rows, ns, x, y, heads);
          e.o = objective(Q, heads, D.H);
          if (!finite_compound(e.o, heads, D.H)) continue;
          e.c = violation(Q, heads);
          /* insert if the queue has room or e beats the worst entry */
          if (qn < Q->k || lex_better(&e, &qv[qn - 1])) {
            uint64_t p = qn < Q->k ? qn : Q->k - 1;
            while (p > 0 && lex_better(&e, &qv[p - 1])) {
              qv[p] = qv[p - 1];
              p--;
            }
            qv[p] = e;
            if (qn < Q->k) qn++;
          }
        }
  }
  uint64_t m = 0;
  for (uint64_t q = 0; q < qn; q++) {
    if (qv[q].c < 0.0 && !keep_violators) continue; /* remove violators at the end */
    out_ids[m] = qv[q].id;
    out_o[m] = qv[q].o;
    if (out_c) out_c[m] = qv[q].c;
    m++;
  }
  *n_out = m;
  free(qv);
  free(x);
  free(y);
  free(heads);
  dec64_free(&D);
  free(slot_base);
  free(row_base);
  free(offset);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Associative embeddings (Section 4.2, eq. "assoc_embeds"): every R-group r  */
/* (a reaction's slot) has a key matrix K_r (d x dU) and every synthon s a     */
/* value vector v_s (dU); the table row of (r, s) is u_{r,s} = K_r v_s. Rows   */
/* are produced in (reaction, slot, synthon) order, the order the library     */
/* tables use. keys: [n_slot_total][d][dU], values: [rows][dU] (float32),      */
/* out: [rows][d] (double). Plain loops, the sum over the value index in      */
/* ascending order.                                                           */
/* ------------------------------------------------------------------------ */
int orc_assoc_embeddings(uint32_t n_reactions, const uint32_t* n_slots, const uint32_t* slot_sizes, uint32_t d,
                         uint32_t dU, const float* keys, const float* values, double* out) {
  uint64_t slot = 0, row = 0;
  for (uint32_t t = 0; t < n_reactions; t++) {
    for (uint32_t s = 0; s < n_slots[t]; s++, slot++) {
      const float* K = keys + slot * (uint64_t)d * dU;
      for (uint32_t i = 0; i < slot_sizes[slot]; i++, row++) {
        const float* v = values + row * dU;
        for (uint32_t j = 0; j < d; j++) {
          double u = 0.0;
          for (uint32_t k = 0; k < dU; k++) u += (double)K[(uint64_t)j * dU + k] * (double)v[k];
          out[row * d + j] = u;
        }
      }
    }
  }
  return 0;
}
