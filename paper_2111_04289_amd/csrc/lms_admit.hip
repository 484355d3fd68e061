// Micro-batch admission control (ConstructMicroBatch, Algorithm 1 of the
// paper) with the latency estimate of Eq. 6 and the running metrics of
// Eq. 4-5.  Host-only: the serving loop calls it every poll.
//
//   EstMaxLat_i = max_j Buff_(i,j) + (sum_j Part_(i,j)) / AvgThPut_(i-1)      (Eq. 6)
//   AvgThPut_i  = (sum of rows of batches 0..i) / (sum of their Proc)          (Eq. 4)
//   MaxLat_i    = max_j Buff_(i,j) + Proc_i                                    (Eq. 5)
//
// Sliding windows (SlideTime > 0) admit the buffered datasets once
// EstMaxLat + poll period >= SlideTime; tumbling windows once it reaches the
// mean MaxLat of the batches completed so far (Eq. 2-3).  The first batch is
// admitted as soon as it holds data; until a batch has completed, AvgThPut is
// undefined and the estimate is the buffering time alone.  A deadline set
// explicitly replaces SlideTime (queries without a window).  With poll_idle
// the test also runs on polls that bring no new data, so a gap in arrivals
// cannot hold buffered data past its deadline.
//
// Learned sizing (lms_admit_set_model): Eq. 6's processing term becomes the
// learned cost model's predicted time of the query's operation chain on a
// micro-batch of the buffered size (each operation on the device MapDevice
// picks with the learned costs), scaled by the ratio of measured to predicted
// processing time over the completed batches.  The model supplies the shape
// of processing time against batch size -- fixed launch and transfer costs,
// which make small batches slower per row than AvgThPut's single rate says --
// and the measured ratio its level on this machine and load.
#include <algorithm>
#include <cmath>
#include <deque>
#include <vector>

#include "lms_internal.h"

namespace lms {
int plan_learned(const lms_op_desc* ops, int32_t nops, const lms_batch_stats* st, const lms_cost_params* cp,
                 int32_t* out_dev, double* out_cost);
}

struct lms_admit {
  lms_admit_params p;
  struct Ds {
    double arrival;
    int64_t rows;
  };
  std::deque<Ds> buffered;  // bufferedFiles, in creation order
  int64_t buffered_rows = 0;
  int64_t batches_done = 0;
  int64_t rows_done = 0;
  double proc_done = 0.0;
  double maxlat_sum = 0.0;
  int64_t admitted = 0;
  // learned sizing
  bool learned = false;
  lms_mlp_model model;
  std::vector<lms_op_desc> ops;
  lms_batch_stats st{};
  double bytes_per_row = 0.0;
  double pred_done = 0.0;  // predicted processing time of the completed batches
  double meas_done = 0.0;  // their measured processing time (those with a prediction)
};

namespace {

// Predicted processing time (ms) of the operation chain on `rows` rows.
double predict_ms(const lms_admit* a, int64_t rows) {
  lms_batch_stats st = a->st;
  st.rows = rows;
  st.batch_bytes = (int64_t)std::llround(a->bytes_per_row * (double)rows);
  if (st.distinct_keys <= 0 || st.distinct_keys > rows) st.distinct_keys = std::max<int64_t>(1, rows);
  lms_cost_params cp{153600.0, 0.1, LMS_PLAN_LEARNED, 0, &a->model};
  std::vector<int32_t> dev(a->ops.size());
  std::vector<double> cost(a->ops.size());
  if (lms::plan_learned(a->ops.data(), (int32_t)a->ops.size(), &st, &cp, dev.data(), cost.data()) != LMS_OK)
    return 0.0;
  double t = 0.0;
  for (double c : cost) t += c;
  return t;
}

// Eq. 6's processing term for `rows` buffered rows; `known` is false while
// nothing has completed (Eq. 4 undefined; the learned form then trusts the
// model at ratio 1).
double proc_term(const lms_admit* a, int64_t rows, bool* known) {
  if (a->learned) {
    *known = true;
    const double ratio = a->pred_done > 0.0 ? a->meas_done / a->pred_done : 1.0;
    return ratio * predict_ms(a, rows);
  }
  *known = a->batches_done > 0 && a->proc_done > 0.0;
  return *known ? (double)rows * a->proc_done / (double)a->rows_done : 0.0;
}

}  // namespace


using namespace lms;

extern "C" int lms_admit_create(const lms_admit_params* p, lms_admit** out) {
  if (!p || !out) return set_error(LMS_EINVAL, "NULL argument");
  *out = nullptr;
  if (p->slide_ms < 0 || p->poll_ms < 0 || p->deadline_ms < 0)
    return set_error(LMS_EINVAL, "negative time parameter");
  lms_admit* a = new lms_admit{};
  a->p = *p;
  *out = a;
  return LMS_OK;
}

extern "C" void lms_admit_free(lms_admit* a) { delete a; }

extern "C" int lms_admit_poll(lms_admit* a, double now_ms, int64_t n_new, const double* arrival_ms,
                              const int64_t* rows, lms_admit_decision* out) {
  if (!a || !out || n_new < 0 || (n_new > 0 && (!arrival_ms || !rows))) return set_error(LMS_EINVAL, "bad arguments");
  *out = lms_admit_decision{};
  // newFiles, sorted by creation time, join the buffered ones
  std::vector<lms_admit::Ds> fresh((size_t)n_new);
  for (int64_t j = 0; j < n_new; ++j) {
    if (rows[j] < 0) return set_error(LMS_EINVAL, "negative row count");
    fresh[(size_t)j] = {arrival_ms[j], rows[j]};
  }
  std::stable_sort(fresh.begin(), fresh.end(), [](const auto& x, const auto& y) { return x.arrival < y.arrival; });
  for (const auto& d : fresh) {
    a->buffered.push_back(d);
    a->buffered_rows += d.rows;
  }
  if (a->buffered.empty() || (n_new == 0 && !a->p.poll_idle)) return LMS_OK;  // keep polling
  double oldest = a->buffered.front().arrival;
  for (const auto& d : a->buffered) oldest = std::min(oldest, d.arrival);
  const double buff = std::max(0.0, now_ms - oldest);
  // deadline: explicit, else SlideTime, else (tumbling) the mean past MaxLat
  bool have_thput = false;
  const double proc = proc_term(a, a->buffered_rows, &have_thput);
  double bound = 0.0;
  if (a->p.deadline_ms > 0) bound = a->p.deadline_ms;
  else if (a->p.slide_ms > 0) bound = a->p.slide_ms;
  else if (a->batches_done > 0) bound = a->maxlat_sum / (double)a->batches_done;
  // Eq. 6; before any batch completed the analytic processing term is unknown and omitted
  const double est = buff + (have_thput ? proc : 0.0);
  const bool admit = a->admitted == 0 || est + a->p.poll_ms >= bound;
  out->est_maxlat_ms = est;
  out->buffered_datasets = (int64_t)a->buffered.size();
  out->buffered_rows = a->buffered_rows;
  if (!admit) return LMS_OK;
  out->admit = 1;
  out->datasets = (int64_t)a->buffered.size();
  out->rows = a->buffered_rows;
  out->oldest_arrival_ms = oldest;
  a->buffered.clear();
  a->buffered_rows = 0;
  ++a->admitted;
  return LMS_OK;
}

extern "C" int lms_admit_done(lms_admit* a, int64_t rows, double proc_ms, double maxlat_ms) {
  if (!a || rows < 0 || proc_ms < 0 || maxlat_ms < 0) return set_error(LMS_EINVAL, "bad arguments");
  ++a->batches_done;
  a->rows_done += rows;
  a->proc_done += proc_ms;
  a->maxlat_sum += maxlat_ms;
  if (a->learned) {
    a->pred_done += predict_ms(a, rows);
    a->meas_done += proc_ms;
  }
  return LMS_OK;
}

extern "C" int lms_admit_set_model(lms_admit* a, const lms_mlp_model* model, const lms_op_desc* ops, int32_t nops,
                                   const lms_batch_stats* per_batch, double bytes_per_row) {
  if (!a) return set_error(LMS_EINVAL, "NULL controller");
  if (!model) {
    a->learned = false;
    return LMS_OK;
  }
  if (!ops || nops <= 0 || !per_batch || bytes_per_row < 0) return set_error(LMS_EINVAL, "bad learned-sizing arguments");
  a->model = *model;
  a->ops.assign(ops, ops + nops);
  a->st = *per_batch;
  a->bytes_per_row = bytes_per_row;
  a->pred_done = 0.0;
  a->meas_done = 0.0;
  a->learned = true;
  return LMS_OK;
}

extern "C" double lms_admit_predict_ms(const lms_admit* a, int64_t rows) {
  if (!a || rows < 0) return -1.0;
  bool known = false;
  const double t = proc_term(a, rows, &known);
  return known ? t : 0.0;
}

extern "C" int lms_admit_get_stats(const lms_admit* a, lms_admit_stats* out) {
  if (!a || !out) return set_error(LMS_EINVAL, "NULL argument");
  out->batches_done = a->batches_done;
  out->admitted = a->admitted;
  out->rows_done = a->rows_done;
  out->buffered_rows = a->buffered_rows;
  out->avg_thput_rows_per_ms = a->proc_done > 0 ? (double)a->rows_done / a->proc_done : 0.0;
  out->mean_maxlat_ms = a->batches_done > 0 ? a->maxlat_sum / (double)a->batches_done : 0.0;
  return LMS_OK;
}
