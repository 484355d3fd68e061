/*
 * lms_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU implementation of what the micro-batch
 * operators compute, used to check the GPU library.  Only the test suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product path never does.  It shares no code, header or constant with the
 * GPU library: it works from the definitions below, not from panes, hash
 * tables or partitions.
 *
 * Operations follow the paper's Table II (Filtering, Projection,
 * Aggregation (Hash) with Expand, Join (Hash)) with the window semantics of
 * Table I (SlideTime; 0 = tumbling) and the range/slide windows of Table III.
 *
 * Definitions (the same ones the library header states):
 *   value of an integer column: int64; of a float column: double.
 *   predicate: integer column `v op ival`, float column `v op fval` (C/IEEE
 *              comparison, so NaN satisfies only !=).  A row passes iff all
 *              predicates hold.
 *   projection: (src * mul + add) in 64-bit two's complement, truncated to the
 *               width of the source column.
 *   window: starts s = origin + k*S for all integers k, S = slide (or len when
 *           slide == 0); a row belongs to every window with s <= ts < s + len.
 *   aggregates per (key, window) over the member rows that pass: COUNT, SUM
 *           (int64, wrapping), MIN, MAX (int64), AVG = (double sum in row
 *           order) / count.
 *   join: for each probe row i in order and each build row j in order with
 *         equal key, the pair (i, payload_j).
 *
 * Parity pins for this file live in tests/ (brute-force loops, library
 * cross-checks and invariants); see the test modules for each function.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { ORC_I32 = 0, ORC_I64 = 1, ORC_F32 = 2, ORC_F64 = 3 };
enum { ORC_LT = 0, ORC_LE = 1, ORC_GT = 2, ORC_GE = 3, ORC_EQ = 4, ORC_NE = 5 };
enum { ORC_COUNT = 0, ORC_SUM = 1, ORC_MIN = 2, ORC_MAX = 3, ORC_AVG = 4 };

static int is_int(int dt) { return dt == ORC_I32 || dt == ORC_I64; }

static int64_t get_int(const void* p, int dt, int64_t i) {
  if (dt == ORC_I32) return ((const int32_t*)p)[i];
  return ((const int64_t*)p)[i];
}

static double get_dbl(const void* p, int dt, int64_t i) {
  switch (dt) {
    case ORC_I32: return (double)((const int32_t*)p)[i];
    case ORC_I64: return (double)((const int64_t*)p)[i];
    case ORC_F32: return (double)((const float*)p)[i];
    default: return ((const double*)p)[i];
  }
}

/* Floor division for b > 0. */
static int64_t floor_div(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b) != 0 && a < 0) q -= 1;
  return q;
}

typedef struct {
  int64_t n;
  int ncols;
  const void* const* cols;
  const int* dt;
  int npred;
  const int* pcol;
  const int* pop;
  const int64_t* pival;
  const double* pfval;
  int nproj;
  const int* prsrc;
  const int64_t* prmul;
  const int64_t* pradd;
} orc_query;

static int cmp_i(int64_t v, int op, int64_t c) {
  switch (op) {
    case ORC_LT: return v < c;
    case ORC_LE: return v <= c;
    case ORC_GT: return v > c;
    case ORC_GE: return v >= c;
    case ORC_EQ: return v == c;
    default: return v != c;
  }
}

static int cmp_f(double v, int op, double c) {
  switch (op) {
    case ORC_LT: return v < c;
    case ORC_LE: return v <= c;
    case ORC_GT: return v > c;
    case ORC_GE: return v >= c;
    case ORC_EQ: return v == c;
    default: return v != c;
  }
}

/* Does row i satisfy every predicate? */
static int passes(const orc_query* q, int64_t i) {
  for (int k = 0; k < q->npred; ++k) {
    int c = q->pcol[k];
    int ok = is_int(q->dt[c]) ? cmp_i(get_int(q->cols[c], q->dt[c], i), q->pop[k], q->pival[k])
                              : cmp_f(get_dbl(q->cols[c], q->dt[c], i), q->pop[k], q->pfval[k]);
    if (!ok) return 0;
  }
  return 1;
}

/* Projection j of row i, as int64 (already truncated to the source width). */
static int64_t proj_value(const orc_query* q, int j, int64_t i) {
  int s = q->prsrc[j];
  uint64_t raw = (uint64_t)get_int(q->cols[s], q->dt[s], i) * (uint64_t)q->prmul[j] + (uint64_t)q->pradd[j];
  if (q->dt[s] == ORC_I32) return (int64_t)(int32_t)(uint32_t)raw;
  return (int64_t)raw;
}

/* Column c of the extended row (input columns, then projections). */
static int ext_is_int(const orc_query* q, int c) { return c >= q->ncols ? 1 : is_int(q->dt[c]); }
static int64_t ext_int(const orc_query* q, int c, int64_t i) {
  return c >= q->ncols ? proj_value(q, c - q->ncols, i) : get_int(q->cols[c], q->dt[c], i);
}
static double ext_dbl(const orc_query* q, int c, int64_t i) {
  return c >= q->ncols ? (double)proj_value(q, c - q->ncols, i) : get_dbl(q->cols[c], q->dt[c], i);
}

/* ---- Filtering + Projection --------------------------------------------
 * Appends, for each passing row in input order, keep[] columns then the
 * projections.  Output column j is int64 for projections and for integer
 * kept columns, double for float kept columns.  Returns the row count. */
int64_t orc_filter_project(int64_t n, int ncols, const void* const* cols, const int* dt, int npred,
                           const int* pcol, const int* pop, const int64_t* pival, const double* pfval, int nkeep,
                           const int* keep, int nproj, const int* prsrc, const int64_t* prmul,
                           const int64_t* pradd, void* const* out) {
  orc_query q = {n, ncols, cols, dt, npred, pcol, pop, pival, pfval, nproj, prsrc, prmul, pradd};
  int64_t m = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (!passes(&q, i)) continue;
    for (int j = 0; j < nkeep; ++j) {
      int c = keep[j];
      if (is_int(dt[c])) ((int64_t*)out[j])[m] = get_int(cols[c], dt[c], i);
      else ((double*)out[j])[m] = get_dbl(cols[c], dt[c], i);
    }
    for (int j = 0; j < nproj; ++j) ((int64_t*)out[nkeep + j])[m] = proj_value(&q, j, i);
    ++m;
  }
  return m;
}

/* ---- Windowed group-by -------------------------------------------------- */

typedef struct {
  int64_t wstart;
  int64_t key;
  int64_t row;
} orc_member; /* one (window, key, row) membership */

static int member_cmp(const void* a, const void* b) {
  const orc_member* x = (const orc_member*)a;
  const orc_member* y = (const orc_member*)b;
  if (x->wstart != y->wstart) return x->wstart < y->wstart ? -1 : 1;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  if (x->row != y->row) return x->row < y->row ? -1 : 1;
  return 0;
}

/* Every window start s (s = origin + k*S) with s <= ts < s + len, visited from
 * the latest start backwards.  Returns how many were written to ws (at most
 * max_out); the total number of such windows is returned through *total. */
static int64_t windows_of(int64_t ts, int64_t len, int64_t S, int64_t origin, int64_t* ws, int64_t max_out,
                          int64_t* total) {
  int64_t k = floor_div(ts - origin, S);
  int64_t m = 0;
  for (; origin + k * S + len > ts; --k) {
    if (m < max_out) ws[m] = origin + k * S;
    ++m;
  }
  *total = m;
  return m < max_out ? m : max_out;
}

/* Computes every (key, window) group with at least one passing row, sorted by
 * (window start, key).  Writes min(groups, cap) groups: out_key, out_ws, and
 * for aggregate a the column out_i + a*cap (COUNT/SUM/MIN/MAX) or out_f + a*cap
 * (AVG).  Returns the number of groups, or -1 if memory ran out. */
int64_t orc_window_agg(int64_t n, int ncols, const void* const* cols, const int* dt, int npred, const int* pcol,
                       const int* pop, const int64_t* pival, const double* pfval, int nproj, const int* prsrc,
                       const int64_t* prmul, const int64_t* pradd, int key_col, int ts_col, int64_t len,
                       int64_t slide, int64_t origin, int nagg, const int* afn, const int* acol, int64_t cap,
                       int64_t* out_key, int64_t* out_ws, int64_t* out_i, double* out_f) {
  orc_query q = {n, ncols, cols, dt, npred, pcol, pop, pival, pfval, nproj, prsrc, prmul, pradd};
  int64_t S = slide == 0 ? len : slide;
  int64_t per_row = len / S + 2;
  int64_t* wbuf = (int64_t*)malloc((size_t)per_row * sizeof(int64_t));
  if (!wbuf) return -1;

  /* Count memberships, then list them. */
  int64_t nm = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (!passes(&q, i)) continue;
    int64_t total;
    windows_of(get_int(cols[ts_col], dt[ts_col], i), len, S, origin, wbuf, 0, &total);
    nm += total;
  }
  orc_member* mem = (orc_member*)malloc((size_t)(nm > 0 ? nm : 1) * sizeof(orc_member));
  if (!mem) {
    free(wbuf);
    return -1;
  }
  int64_t m = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (!passes(&q, i)) continue;
    int64_t total;
    int64_t got = windows_of(get_int(cols[ts_col], dt[ts_col], i), len, S, origin, wbuf, per_row, &total);
    int64_t key = get_int(cols[key_col], dt[key_col], i);
    for (int64_t w = 0; w < got; ++w) {
      mem[m].wstart = wbuf[w];
      mem[m].key = key;
      mem[m].row = i;
      ++m;
    }
  }
  free(wbuf);
  qsort(mem, (size_t)nm, sizeof(orc_member), member_cmp);

  /* One pass over runs of equal (window, key); rows of a run are in row order. */
  int64_t g = 0;
  for (int64_t a = 0; a < nm;) {
    int64_t b = a;
    while (b < nm && mem[b].wstart == mem[a].wstart && mem[b].key == mem[a].key) ++b;
    if (g < cap) {
      out_key[g] = mem[a].key;
      out_ws[g] = mem[a].wstart;
      for (int k = 0; k < nagg; ++k) {
        int c = acol[k];
        int64_t cnt = b - a;
        if (afn[k] == ORC_COUNT) {
          out_i[k * cap + g] = cnt;
        } else if (afn[k] == ORC_AVG) {
          double s = 0.0;
          for (int64_t r = a; r < b; ++r) s += ext_dbl(&q, c, mem[r].row);
          out_f[k * cap + g] = s / (double)cnt;
        } else {
          uint64_t s = 0;
          int64_t mn = ext_int(&q, c, mem[a].row), mx = mn;
          for (int64_t r = a; r < b; ++r) {
            int64_t v = ext_int(&q, c, mem[r].row);
            s += (uint64_t)v;
            if (v < mn) mn = v;
            if (v > mx) mx = v;
          }
          out_i[k * cap + g] = afn[k] == ORC_SUM ? (int64_t)s : (afn[k] == ORC_MIN ? mn : mx);
        }
      }
    }
    ++g;
    a = b;
  }
  free(mem);
  (void)ext_is_int;
  return g;
}

/* Aggregates of the single group (qkey, qws) by a scan of every row: the
 * definition applied to one output, used to check sampled groups of large
 * batches.  Returns the group's COUNT (0 if the window start is not aligned
 * or holds no passing row of the key). */
int64_t orc_window_group(int64_t n, int ncols, const void* const* cols, const int* dt, int npred, const int* pcol,
                         const int* pop, const int64_t* pival, const double* pfval, int nproj, const int* prsrc,
                         const int64_t* prmul, const int64_t* pradd, int key_col, int ts_col, int64_t len,
                         int64_t slide, int64_t origin, int nagg, const int* afn, const int* acol, int64_t qkey,
                         int64_t qws, int64_t* out_i, double* out_f) {
  orc_query q = {n, ncols, cols, dt, npred, pcol, pop, pival, pfval, nproj, prsrc, prmul, pradd};
  int64_t S = slide == 0 ? len : slide;
  if (floor_div(qws - origin, S) * S != qws - origin) return 0;
  int64_t cnt = 0;
  for (int k = 0; k < nagg; ++k) {
    out_i[k] = 0;
    out_f[k] = 0.0;
  }
  uint64_t* sums = (uint64_t*)calloc((size_t)(nagg > 0 ? nagg : 1), sizeof(uint64_t));
  double* fs = (double*)calloc((size_t)(nagg > 0 ? nagg : 1), sizeof(double));
  for (int64_t i = 0; i < n; ++i) {
    if (get_int(cols[key_col], dt[key_col], i) != qkey) continue;
    int64_t ts = get_int(cols[ts_col], dt[ts_col], i);
    if (!(qws <= ts && ts < qws + len)) continue;
    if (!passes(&q, i)) continue;
    for (int k = 0; k < nagg; ++k) {
      int c = acol[k];
      if (afn[k] == ORC_COUNT) continue;
      if (afn[k] == ORC_AVG) {
        fs[k] += ext_dbl(&q, c, i);
        continue;
      }
      int64_t v = ext_int(&q, c, i);
      sums[k] += (uint64_t)v;
      if (cnt == 0 || (afn[k] == ORC_MIN && v < out_i[k]) || (afn[k] == ORC_MAX && v > out_i[k])) out_i[k] = v;
    }
    ++cnt;
  }
  for (int k = 0; k < nagg; ++k) {
    if (afn[k] == ORC_COUNT) out_i[k] = cnt;
    else if (afn[k] == ORC_SUM) out_i[k] = (int64_t)sums[k];
    else if (afn[k] == ORC_AVG) out_f[k] = cnt ? fs[k] / (double)cnt : 0.0;
  }
  free(sums);
  free(fs);
  return cnt;
}

typedef struct {
  int64_t l, a;
} orc_brow_pair;

static int pair_cmp(const void* x, const void* y) {
  const orc_brow_pair* p = (const orc_brow_pair*)x;
  const orc_brow_pair* q = (const orc_brow_pair*)y;
  if (p->l != q->l) return p->l < q->l ? -1 : 1;
  if (p->a != q->a) return p->a < q->a ? -1 : 1;
  return 0;
}

/* ---- Windowed group-by over a composite key ------------------------------
 * Table III's LR2S groups by (highway, direction, segment): the group key is
 * the tuple of nkey integer columns.  Same definition as orc_window_agg with
 * the tuple in place of the single key: every passing row joins each window
 * holding its event time; groups are sorted by (window start, key tuple).
 * out_keys holds key column j of group g at out_keys[j*cap + g]. */

typedef struct {
  int64_t wstart;
  int64_t key[4];
  int64_t row;
} orc_tmember;

static int g_tnkey; /* tuple width for tmember_cmp (the oracle is single-threaded) */

static int tmember_cmp(const void* a, const void* b) {
  const orc_tmember* x = (const orc_tmember*)a;
  const orc_tmember* y = (const orc_tmember*)b;
  if (x->wstart != y->wstart) return x->wstart < y->wstart ? -1 : 1;
  for (int j = 0; j < g_tnkey; ++j)
    if (x->key[j] != y->key[j]) return x->key[j] < y->key[j] ? -1 : 1;
  if (x->row != y->row) return x->row < y->row ? -1 : 1;
  return 0;
}

static int same_group(const orc_tmember* x, const orc_tmember* y, int nkey) {
  if (x->wstart != y->wstart) return 0;
  for (int j = 0; j < nkey; ++j)
    if (x->key[j] != y->key[j]) return 0;
  return 1;
}

int64_t orc_window_agg_keys(int64_t n, int ncols, const void* const* cols, const int* dt, int npred,
                            const int* pcol, const int* pop, const int64_t* pival, const double* pfval, int nproj,
                            const int* prsrc, const int64_t* prmul, const int64_t* pradd, int nkey,
                            const int* key_cols, int ts_col, int64_t len, int64_t slide, int64_t origin, int nagg,
                            const int* afn, const int* acol, int64_t cap, int64_t* out_keys, int64_t* out_ws,
                            int64_t* out_i, double* out_f) {
  orc_query q = {n, ncols, cols, dt, npred, pcol, pop, pival, pfval, nproj, prsrc, prmul, pradd};
  if (nkey < 1 || nkey > 4) return -2;
  int64_t S = slide == 0 ? len : slide;
  int64_t per_row = len / S + 2;
  int64_t* wbuf = (int64_t*)malloc((size_t)per_row * sizeof(int64_t));
  if (!wbuf) return -1;
  int64_t nm = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (!passes(&q, i)) continue;
    int64_t total;
    windows_of(get_int(cols[ts_col], dt[ts_col], i), len, S, origin, wbuf, 0, &total);
    nm += total;
  }
  orc_tmember* mem = (orc_tmember*)malloc((size_t)(nm > 0 ? nm : 1) * sizeof(orc_tmember));
  if (!mem) {
    free(wbuf);
    return -1;
  }
  int64_t m = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (!passes(&q, i)) continue;
    int64_t total;
    int64_t got = windows_of(get_int(cols[ts_col], dt[ts_col], i), len, S, origin, wbuf, per_row, &total);
    for (int64_t w = 0; w < got; ++w) {
      mem[m].wstart = wbuf[w];
      for (int j = 0; j < 4; ++j) mem[m].key[j] = j < nkey ? get_int(cols[key_cols[j]], dt[key_cols[j]], i) : 0;
      mem[m].row = i;
      ++m;
    }
  }
  free(wbuf);
  g_tnkey = nkey;
  qsort(mem, (size_t)nm, sizeof(orc_tmember), tmember_cmp);
  int64_t g = 0;
  for (int64_t a = 0; a < nm;) {
    int64_t b = a;
    while (b < nm && same_group(&mem[b], &mem[a], nkey)) ++b;
    if (g < cap) {
      for (int j = 0; j < nkey; ++j) out_keys[j * cap + g] = mem[a].key[j];
      out_ws[g] = mem[a].wstart;
      for (int k = 0; k < nagg; ++k) {
        int c = acol[k];
        int64_t cnt = b - a;
        if (afn[k] == ORC_COUNT) {
          out_i[k * cap + g] = cnt;
        } else if (afn[k] == ORC_AVG) {
          double s = 0.0;
          for (int64_t r = a; r < b; ++r) s += ext_dbl(&q, c, mem[r].row);
          out_f[k * cap + g] = s / (double)cnt;
        } else {
          uint64_t s = 0;
          int64_t mn = ext_int(&q, c, mem[a].row), mx = mn;
          for (int64_t r = a; r < b; ++r) {
            int64_t v = ext_int(&q, c, mem[r].row);
            s += (uint64_t)v;
            if (v < mn) mn = v;
            if (v > mx) mx = v;
          }
          out_i[k * cap + g] = afn[k] == ORC_SUM ? (int64_t)s : (afn[k] == ORC_MIN ? mn : mx);
        }
      }
    }
    ++g;
    a = b;
  }
  free(mem);
  return g;
}

/* ---- Windowed self-join ---------------------------------------------------
 * Table III's LR1 joins the stream with the rows of its own range/slide window
 * on equal keys (A.vehicle == L.vehicle).  Read per micro-batch: for every
 * window and every ordered pair of passing rows (l, a) that both lie in the
 * window and have equal keys (l == a included), one output (window start, l,
 * a).  Listed in (window start, l, a) order.  Writes min(pairs, cap); returns
 * the number of pairs, or -1 if memory ran out. */
int64_t orc_window_self_join(int64_t n, int ncols, const void* const* cols, const int* dt, int npred,
                             const int* pcol, const int* pop, const int64_t* pival, const double* pfval,
                             int key_col, int ts_col, int64_t len, int64_t slide, int64_t origin, int64_t cap,
                             int64_t* out_ws, int64_t* out_l, int64_t* out_a) {
  orc_query q = {n, ncols, cols, dt, npred, pcol, pop, pival, pfval, 0, NULL, NULL, NULL};
  int64_t S = slide == 0 ? len : slide;
  int64_t per_row = len / S + 2;
  int64_t* wbuf = (int64_t*)malloc((size_t)per_row * sizeof(int64_t));
  if (!wbuf) return -1;
  int64_t nm = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (!passes(&q, i)) continue;
    int64_t total;
    windows_of(get_int(cols[ts_col], dt[ts_col], i), len, S, origin, wbuf, 0, &total);
    nm += total;
  }
  orc_member* mem = (orc_member*)malloc((size_t)(nm > 0 ? nm : 1) * sizeof(orc_member));
  if (!mem) {
    free(wbuf);
    return -1;
  }
  int64_t m = 0;
  for (int64_t i = 0; i < n; ++i) {
    if (!passes(&q, i)) continue;
    int64_t total;
    int64_t got = windows_of(get_int(cols[ts_col], dt[ts_col], i), len, S, origin, wbuf, per_row, &total);
    for (int64_t w = 0; w < got; ++w) {
      mem[m].wstart = wbuf[w];
      mem[m].key = get_int(cols[key_col], dt[key_col], i);
      mem[m].row = i;
      ++m;
    }
  }
  free(wbuf);
  /* members sorted by (window, key, row): each run of equal (window, key) is a
   * window's rows of one key in row order, and its pairs are the run squared.
   * A window's pairs are collected, then sorted into (l, a) order. */
  qsort(mem, (size_t)nm, sizeof(orc_member), member_cmp);
  int64_t g = 0;
  int64_t pcap = 1024;
  orc_brow_pair* pairs = (orc_brow_pair*)malloc((size_t)pcap * sizeof(orc_brow_pair));
  if (!pairs) {
    free(mem);
    return -1;
  }
  for (int64_t a = 0; a < nm;) {
    int64_t wend = a;
    while (wend < nm && mem[wend].wstart == mem[a].wstart) ++wend;
    int64_t c = 0;
    for (int64_t r = a; r < wend;) {
      int64_t e = r;
      while (e < wend && mem[e].key == mem[r].key) ++e;
      for (int64_t x = r; x < e; ++x)
        for (int64_t y = r; y < e; ++y) {
          if (c == pcap) {
            orc_brow_pair* grown = (orc_brow_pair*)realloc(pairs, (size_t)(2 * pcap) * sizeof(orc_brow_pair));
            if (!grown) {
              free(pairs);
              free(mem);
              return -1;
            }
            pairs = grown;
            pcap *= 2;
          }
          pairs[c].l = mem[x].row;
          pairs[c].a = mem[y].row;
          ++c;
        }
      r = e;
    }
    qsort(pairs, (size_t)c, sizeof(orc_brow_pair), pair_cmp);
    for (int64_t k = 0; k < c; ++k, ++g)
      if (g < cap) {
        out_ws[g] = mem[a].wstart;
        out_l[g] = pairs[k].l;
        out_a[g] = pairs[k].a;
      }
    a = wend;
  }
  free(pairs);
  free(mem);
  return g;
}

/* ---- Stream-static join ------------------------------------------------- */

typedef struct {
  int64_t key;
  int64_t row;
} orc_brow;

static int brow_cmp(const void* a, const void* b) {
  const orc_brow* x = (const orc_brow*)a;
  const orc_brow* y = (const orc_brow*)b;
  if (x->key != y->key) return x->key < y->key ? -1 : 1;
  if (x->row != y->row) return x->row < y->row ? -1 : 1;
  return 0;
}

/* Pairs (i, payload_j) for probe rows i in order and equal-key build rows j in
 * order.  The build side is sorted by (key, row) so that the equal-key rows of
 * each probe key are found by binary search; the emitted order is exactly the
 * (i, j) order of the definition.  Writes min(pairs, cap); returns the number
 * of pairs, or -1 if memory ran out. */
int64_t orc_hash_join(int64_t nb, const void* bkey, int bkey_dt, const int32_t* bpay, int64_t np, const void* pkey,
                      int pkey_dt, int64_t cap, int64_t* out_probe, int32_t* out_pay) {
  orc_brow* rows = (orc_brow*)malloc((size_t)(nb > 0 ? nb : 1) * sizeof(orc_brow));
  if (!rows) return -1;
  for (int64_t j = 0; j < nb; ++j) {
    rows[j].key = get_int(bkey, bkey_dt, j);
    rows[j].row = j;
  }
  qsort(rows, (size_t)nb, sizeof(orc_brow), brow_cmp);
  int64_t m = 0;
  for (int64_t i = 0; i < np; ++i) {
    int64_t k = get_int(pkey, pkey_dt, i);
    int64_t lo = 0, hi = nb; /* first index with rows[idx].key >= k */
    while (lo < hi) {
      int64_t mid = lo + (hi - lo) / 2;
      if (rows[mid].key < k) lo = mid + 1;
      else hi = mid;
    }
    for (int64_t j = lo; j < nb && rows[j].key == k; ++j) {
      if (m < cap) {
        out_probe[m] = i;
        out_pay[m] = bpay[rows[j].row];
      }
      ++m;
    }
  }
  free(rows);
  return m;
}
