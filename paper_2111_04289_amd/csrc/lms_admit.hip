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
#include <algorithm>
#include <deque>
#include <vector>

#include "lms_internal.h"

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
};

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
  const bool have_thput = a->batches_done > 0 && a->proc_done > 0.0;
  double bound = 0.0;
  if (a->p.deadline_ms > 0) bound = a->p.deadline_ms;
  else if (a->p.slide_ms > 0) bound = a->p.slide_ms;
  else if (a->batches_done > 0) bound = a->maxlat_sum / (double)a->batches_done;
  // Eq. 6; before any batch completed the processing term is unknown and omitted
  const double est = buff + (have_thput ? (double)a->buffered_rows * a->proc_done / (double)a->rows_done : 0.0);
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
  return LMS_OK;
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
