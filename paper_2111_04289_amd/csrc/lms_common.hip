// Error reporting, query validation and the MapDevice planner (host code).
#include <stdarg.h>
#include <stdio.h>

#include <atomic>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "lms_internal.h"

namespace lms {

static thread_local std::string g_last_error;

int set_error(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return code;
}

// ---- kernel tracing ----------------------------------------------------------
namespace {
struct TraceRec {
  std::string name;
  hipEvent_t start, stop;
};
std::atomic<int> g_trace_on{0};
std::mutex g_trace_mu;
std::vector<TraceRec> g_trace_recs;     // recorded, not yet read
std::vector<hipEvent_t> g_trace_pool;   // free events
hipEvent_t trace_event() {
  if (!g_trace_pool.empty()) {
    hipEvent_t e = g_trace_pool.back();
    g_trace_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace

TraceScope::TraceScope(const char* name, hipStream_t s) : st(s) {
  if (!g_trace_on.load(std::memory_order_relaxed)) return;
  std::lock_guard<std::mutex> lk(g_trace_mu);
  hipEvent_t a = trace_event(), b = trace_event();
  if (!a || !b) return;
  if (hipEventRecord(a, st) != hipSuccess) return;
  g_trace_recs.push_back(TraceRec{name, a, b});
  slot = (int)g_trace_recs.size() - 1;
}

TraceScope::~TraceScope() {
  if (slot < 0) return;
  std::lock_guard<std::mutex> lk(g_trace_mu);
  if (slot < (int)g_trace_recs.size()) (void)hipEventRecord(g_trace_recs[slot].stop, st);
}

int check_hip(hipError_t e, const char* what) {
  if (e == hipSuccess) return LMS_OK;
  return set_error(LMS_EHIP, "%s: %s", what, hipGetErrorString(e));
}

static bool valid_dtype(int dt) { return dt >= LMS_I32 && dt <= LMS_F64; }
static bool int_dtype(int dt) { return dt == LMS_I32 || dt == LMS_I64; }

int build_query(const lms_batch* in, const lms_pred* preds, int32_t npred, const lms_proj* projs, int32_t nproj,
                Query* q) {
  if (!in) return set_error(LMS_EINVAL, "input batch is NULL");
  if (in->ncols < 0 || in->ncols > kMaxCols) return set_error(LMS_EINVAL, "ncols %d outside [0, %d]", in->ncols, kMaxCols);
  if (in->ncols > 0 && !in->cols) return set_error(LMS_EINVAL, "cols is NULL");
  if (in->nrows < 0) return set_error(LMS_EINVAL, "negative nrows");
  if (npred < 0 || npred > kMaxPreds) return set_error(LMS_EINVAL, "npred %d outside [0, %d]", npred, kMaxPreds);
  if (nproj < 0 || nproj > kMaxProjs) return set_error(LMS_EINVAL, "nproj %d outside [0, %d]", nproj, kMaxProjs);
  if (npred > 0 && !preds) return set_error(LMS_EINVAL, "preds is NULL");
  if (nproj > 0 && !projs) return set_error(LMS_EINVAL, "projs is NULL");
  *q = Query{};
  q->ncols = in->ncols;
  q->nrows = in->nrows;
  for (int c = 0; c < in->ncols; ++c) {
    if (!valid_dtype(in->cols[c].dtype)) return set_error(LMS_EINVAL, "column %d has bad dtype %d", c, in->cols[c].dtype);
    if (in->nrows > 0 && !in->cols[c].data) return set_error(LMS_EINVAL, "column %d data is NULL", c);
    q->col[c] = in->cols[c].data;
    q->dt[c] = in->cols[c].dtype;
  }
  q->npred = npred;
  for (int k = 0; k < npred; ++k) {
    if (preds[k].col < 0 || preds[k].col >= in->ncols)
      return set_error(LMS_EINVAL, "predicate %d column %d out of range", k, preds[k].col);
    if (preds[k].op < LMS_LT || preds[k].op > LMS_NE) return set_error(LMS_EINVAL, "predicate %d bad op", k);
    q->pcol[k] = preds[k].col;
    q->pop[k] = preds[k].op;
    q->pival[k] = preds[k].ival;
    q->pfval[k] = preds[k].fval;
  }
  q->nproj = nproj;
  for (int j = 0; j < nproj; ++j) {
    if (projs[j].src < 0 || projs[j].src >= in->ncols)
      return set_error(LMS_EINVAL, "projection %d source %d out of range", j, projs[j].src);
    if (!int_dtype(in->cols[projs[j].src].dtype))
      return set_error(LMS_EINVAL, "projection %d needs an integer source column", j);
    q->prsrc[j] = projs[j].src;
    q->prmul[j] = projs[j].mul;
    q->pradd[j] = projs[j].add;
  }
  return LMS_OK;
}

}  // namespace lms

using namespace lms;

extern "C" int lms_abi_version(void) { return LMS_ABI_VERSION; }

extern "C" int lms_trace_enable(int32_t on) {
  g_trace_on.store(on ? 1 : 0);
  return LMS_OK;
}

extern "C" int lms_trace_read(lms_trace_stat* out, int32_t max_out) {
  std::vector<TraceRec> recs;
  {
    std::lock_guard<std::mutex> lk(g_trace_mu);
    recs.swap(g_trace_recs);
  }
  std::map<std::string, lms_trace_stat> agg;
  int rc = LMS_OK;
  for (auto& r : recs) {
    float ms = 0.f;
    if (rc == LMS_OK) rc = check_hip(hipEventSynchronize(r.stop), "hipEventSynchronize");
    if (rc == LMS_OK) rc = check_hip(hipEventElapsedTime(&ms, r.start, r.stop), "hipEventElapsedTime");
    auto it = agg.find(r.name);
    if (it == agg.end()) {
      lms_trace_stat st{};
      std::strncpy(st.name, r.name.c_str(), sizeof st.name - 1);
      st.min_ms = ms;
      st.max_ms = ms;
      it = agg.emplace(r.name, st).first;
    }
    it->second.launches += 1;
    it->second.total_ms += ms;
    it->second.min_ms = std::min(it->second.min_ms, (double)ms);
    it->second.max_ms = std::max(it->second.max_ms, (double)ms);
  }
  {
    std::lock_guard<std::mutex> lk(g_trace_mu);
    for (auto& r : recs) {
      g_trace_pool.push_back(r.start);
      g_trace_pool.push_back(r.stop);
    }
  }
  if (rc != LMS_OK) return rc;
  int n = 0;
  for (auto& kv : agg) {
    if (out && n < max_out) out[n] = kv.second;
    ++n;
  }
  return n;
}

extern "C" const char* lms_last_error(void) { return g_last_error.c_str(); }

// Table II of the paper: base cost of each operation kind.
extern "C" double lms_table2_base_cost(int32_t kind) {
  switch (kind) {
    case LMS_OP_AGG:
    case LMS_OP_FILTER:
    case LMS_OP_SHUFFLE: return 1.0;
    case LMS_OP_PROJECT:
    case LMS_OP_JOIN:
    case LMS_OP_EXPAND: return 0.9;
    case LMS_OP_SCAN:
    case LMS_OP_SORT: return 0.8;
    default: return -1.0;
  }
}

namespace lms {
// Learned-placement hook, defined by the MLP module; returns LMS_OK and fills
// out_dev when it handled the request.
int plan_learned(const lms_op_desc* ops, int32_t nops, const lms_batch_stats* st, const lms_cost_params* cp,
                 int32_t* out_dev, double* out_cost) __attribute__((weak));
}  // namespace lms

// MapDevice (Algorithm 2) with Eq. 7-9; see lms.h.
extern "C" int lms_plan(const lms_op_desc* ops, int32_t nops, const lms_batch_stats* st, const lms_cost_params* cp,
                        int32_t* out_dev, double* out_cost) {
  if (nops < 0) return set_error(LMS_EINVAL, "nops < 0");
  if (nops > 0 && (!ops || !out_dev)) return set_error(LMS_EINVAL, "ops/out_dev is NULL");
  if (!st || !cp) return set_error(LMS_EINVAL, "stats/params is NULL");
  if (st->num_cores <= 0) return set_error(LMS_EINVAL, "num_cores must be positive");
  if (st->batch_bytes <= 0) return set_error(LMS_EINVAL, "batch_bytes must be positive");
  if (!(cp->infpt_bytes > 0)) return set_error(LMS_EINVAL, "infpt_bytes must be positive");
  for (int o = 0; o < nops; ++o) {
    double b = ops[o].base_cost > 0 ? ops[o].base_cost : lms_table2_base_cost(ops[o].kind);
    if (!(b > 0)) return set_error(LMS_EINVAL, "operation %d has unknown kind %d", o, ops[o].kind);
  }
  if (cp->mode == LMS_PLAN_LEARNED && cp->model && plan_learned) {
    for (int o = 0; o < nops; ++o) out_dev[o] = LMS_DEV_GPU;
    int rc = plan_learned(ops, nops, st, cp, out_dev, out_cost);
    if (rc == LMS_OK) return rc;
  }
  // Per-core partition size (Sec. III-D) relative to the inflection point.
  const double x = ((double)st->batch_bytes / (double)st->num_cores) / cp->infpt_bytes;
  for (int o = 0; o < nops; ++o) out_dev[o] = LMS_DEV_GPU;  // every operation starts on the GPU
  for (int o = 0; o < nops; ++o) {
    const double base = ops[o].base_cost > 0 ? ops[o].base_cost : lms_table2_base_cost(ops[o].kind);
    double cpu = base * x;                // Eq. 7
    double gpu = base / x;                // Eq. 8
    const double trans = cp->base_trans * x;  // Eq. 9
    if (o == 0 || o == nops - 1 || out_dev[o - 1] == LMS_DEV_CPU) gpu += trans;
    else cpu += trans;
    if (gpu > cpu) out_dev[o] = LMS_DEV_CPU;
    if (out_cost) out_cost[o] = out_dev[o] == LMS_DEV_CPU ? cpu : gpu;
  }
  return LMS_OK;
}

// ---- online inflection-point regression (Eq. 10) ----------------------------
// After each micro-batch the controller records the InfPT it used with the
// batch's throughput (rows per ms) and MaxLat; before the next one it fits
// InfPT = b0 + b1 * Throughput + b2 * Latency by least squares over the last
// `history` records (all if 0) and evaluates it at the targets: the largest
// throughput seen and the target latency.  The regressors are centred and
// scaled before the normal equations are solved, so the 3x3 system stays
// well conditioned; with fewer than three records, collinear regressors or a
// prediction that is not a positive finite number, the last InfPT is kept.
// The value handed out is then multiplied by 1 + jitter * u, u uniform in
// [-1, 1] from SplitMix64 (Steele, Lea and Flood's generator; one draw per
// call): without it every record would carry the same InfPT and the fit
// could never move it.
struct lms_infpt {
  double cur;
  int32_t history;
  double jitter;
  uint64_t rng;
  std::vector<double> x1, x2, y;
};

namespace {
uint64_t splitmix64_next(uint64_t* s) {
  uint64_t z = (*s += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}
}  // namespace

extern "C" int lms_infpt_create(double init_bytes, int32_t history, double jitter, uint64_t seed, lms_infpt** out) {
  if (!out) return set_error(LMS_EINVAL, "out is NULL");
  *out = nullptr;
  if (!(init_bytes > 0) || history < 0 || !(jitter >= 0 && jitter < 1))
    return set_error(LMS_EINVAL, "bad inflection-point tuner parameters");
  *out = new lms_infpt{init_bytes, history, jitter, seed, {}, {}, {}};
  return LMS_OK;
}

extern "C" void lms_infpt_free(lms_infpt* t) { delete t; }

extern "C" int lms_infpt_record(lms_infpt* t, double infpt_used, double thput, double maxlat) {
  if (!t || !(infpt_used > 0) || !(thput >= 0) || !(maxlat >= 0)) return set_error(LMS_EINVAL, "bad record");
  t->x1.push_back(thput);
  t->x2.push_back(maxlat);
  t->y.push_back(infpt_used);
  return LMS_OK;
}

extern "C" double lms_infpt_next(lms_infpt* t, double target_latency) {
  if (!t) return -1.0;
  const size_t n = t->y.size();
  const size_t lo = (t->history > 0 && n > (size_t)t->history) ? n - (size_t)t->history : 0;
  const size_t m = n - lo;
  if (m >= 3) {
    double m1 = 0, m2 = 0, my = 0, tmax = t->x1[0], lsum = 0;
    for (size_t i = 0; i < n; ++i) {
      tmax = std::max(tmax, t->x1[i]);
      lsum += t->x2[i];
    }
    for (size_t i = lo; i < n; ++i) {
      m1 += t->x1[i];
      m2 += t->x2[i];
      my += t->y[i];
    }
    m1 /= (double)m;
    m2 /= (double)m;
    my /= (double)m;
    double s1 = 0, s2 = 0;
    for (size_t i = lo; i < n; ++i) {
      s1 += (t->x1[i] - m1) * (t->x1[i] - m1);
      s2 += (t->x2[i] - m2) * (t->x2[i] - m2);
    }
    s1 = std::sqrt(s1 / (double)m);
    s2 = std::sqrt(s2 / (double)m);
    if (s1 > 0 && s2 > 0) {
      // centred, scaled regressors: the intercept is then the mean of y
      double a11 = 0, a12 = 0, a22 = 0, r1 = 0, r2 = 0;
      for (size_t i = lo; i < n; ++i) {
        const double u = (t->x1[i] - m1) / s1, v = (t->x2[i] - m2) / s2, w = t->y[i] - my;
        a11 += u * u;
        a12 += u * v;
        a22 += v * v;
        r1 += u * w;
        r2 += v * w;
      }
      const double det = a11 * a22 - a12 * a12;
      if (det > 1e-9 * a11 * a22) {
        const double c1 = (r1 * a22 - r2 * a12) / det, c2 = (a11 * r2 - a12 * r1) / det;
        const double lat = target_latency > 0 ? target_latency : lsum / (double)n;
        const double pred = my + c1 * (tmax - m1) / s1 + c2 * (lat - m2) / s2;
        if (std::isfinite(pred) && pred > 0) t->cur = pred;
      }
    }
  }
  const double u = (double)(splitmix64_next(&t->rng) >> 11) * 0x1.0p-53 * 2.0 - 1.0;
  return t->cur * (1.0 + t->jitter * u);
}
