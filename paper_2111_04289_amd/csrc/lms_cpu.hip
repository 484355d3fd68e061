// CPU execution functions of the operators (host code only).
//
// MapDevice (Algorithm 2) places every operation either on the GPU or on the
// CPU cores of the executor (Sec. III-D: one data partition per core).  These
// are the CPU functions: the same semantics as the GPU entry points, on host
// columns, parallel over `nthreads` cores the way the paper's executor splits
// a micro-batch into NumCores partitions (Table I).
//
//  * filter/project: per-thread row ranges, counts, prefix, ordered writes.
//  * windowed group-by: each thread routes its passing rows by key hash to one
//    of nthreads partitions; each partition is aggregated per (key, pane) in a
//    hash map, its keys' panes are sorted and the windows composed.
//  * join: open-addressing build, probe over per-thread row ranges, outputs
//    concatenated in probe order.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>
#include <unordered_map>
#include <vector>

#include "lms_internal.h"

namespace lms {
namespace {

struct HostQuery {
  const lms_batch* in;
  const lms_pred* preds;
  int32_t npred;
  const lms_proj* projs;
  int32_t nproj;
};

inline int64_t h_i64(const lms_col& c, int64_t i) {
  return c.dtype == LMS_I32 ? (int64_t)((const int32_t*)c.data)[i] : ((const int64_t*)c.data)[i];
}
inline double h_f64(const lms_col& c, int64_t i) {
  switch (c.dtype) {
    case LMS_I32: return (double)((const int32_t*)c.data)[i];
    case LMS_I64: return (double)((const int64_t*)c.data)[i];
    case LMS_F32: return (double)((const float*)c.data)[i];
    default: return ((const double*)c.data)[i];
  }
}
template <class T>
inline bool h_cmp(T v, int op, T c) {
  switch (op) {
    case LMS_LT: return v < c;
    case LMS_LE: return v <= c;
    case LMS_GT: return v > c;
    case LMS_GE: return v >= c;
    case LMS_EQ: return v == c;
    default: return v != c;
  }
}
inline bool h_passes(const HostQuery& q, int64_t i) {
  for (int k = 0; k < q.npred; ++k) {
    const lms_col& c = q.in->cols[q.preds[k].col];
    const bool ok = (c.dtype == LMS_I32 || c.dtype == LMS_I64) ? h_cmp<int64_t>(h_i64(c, i), q.preds[k].op, q.preds[k].ival)
                                                              : h_cmp<double>(h_f64(c, i), q.preds[k].op, q.preds[k].fval);
    if (!ok) return false;
  }
  return true;
}
inline int64_t h_proj(const HostQuery& q, int j, int64_t i) {
  const lms_col& c = q.in->cols[q.projs[j].src];
  const uint64_t raw = (uint64_t)h_i64(c, i) * (uint64_t)q.projs[j].mul + (uint64_t)q.projs[j].add;
  return c.dtype == LMS_I32 ? (int64_t)(int32_t)(uint32_t)raw : (int64_t)raw;
}
inline int64_t h_ext_i64(const HostQuery& q, int c, int64_t i) {
  return c < q.in->ncols ? h_i64(q.in->cols[c], i) : h_proj(q, c - q.in->ncols, i);
}
inline double h_ext_f64(const HostQuery& q, int c, int64_t i) {
  return c < q.in->ncols ? h_f64(q.in->cols[c], i) : (double)h_proj(q, c - q.in->ncols, i);
}

template <class F>
void parallel_for(int nthreads, F f) {
  if (nthreads <= 1) {
    f(0);
    return;
  }
  std::vector<std::thread> ts;
  ts.reserve(nthreads);
  for (int t = 0; t < nthreads; ++t) ts.emplace_back(f, t);
  for (auto& t : ts) t.join();
}

inline int64_t range_lo(int64_t n, int t, int T) { return n * t / T; }

struct Acc {
  uint64_t cnt = 0;
  uint64_t v[kMaxAggs];
};

struct PaneKey {
  int64_t key, pane;
  bool operator==(const PaneKey& o) const { return key == o.key && pane == o.pane; }
};
struct PaneKeyHash {
  size_t operator()(const PaneKey& k) const { return (size_t)fmix64((uint64_t)k.key ^ fmix64((uint64_t)k.pane)); }
};

}  // namespace
}  // namespace lms

using namespace lms;

extern "C" int lms_cpu_filter_project(const lms_batch* in, const lms_pred* preds, int32_t npred, const int32_t* keep,
                                      int32_t nkeep, const lms_proj* projs, int32_t nproj, const lms_batch* out,
                                      int64_t* count, int32_t nthreads) {
  Query dummy;
  int rc = build_query(in, preds, npred, projs, nproj, &dummy);
  if (rc) return rc;
  if (!out || out->ncols != nkeep + nproj || !count) return set_error(LMS_EINVAL, "bad output batch / count");
  if (nkeep > 0 && !keep) return set_error(LMS_EINVAL, "keep is NULL");
  for (int j = 0; j < nkeep; ++j)
    if (keep[j] < 0 || keep[j] >= in->ncols || out->cols[j].dtype != in->cols[keep[j]].dtype)
      return set_error(LMS_EINVAL, "keep column %d invalid", j);
  for (int j = 0; j < nproj; ++j)
    if (out->cols[nkeep + j].dtype != in->cols[projs[j].src].dtype)
      return set_error(LMS_EINVAL, "projection output %d has the wrong dtype", j);
  const int T = std::max(1, nthreads);
  const int64_t n = in->nrows;
  HostQuery q{in, preds, npred, projs, nproj};
  std::vector<int64_t> cnt(T + 1, 0);
  parallel_for(T, [&](int t) {
    int64_t c = 0;
    for (int64_t i = range_lo(n, t, T); i < range_lo(n, t + 1, T); ++i) c += h_passes(q, i);
    cnt[t + 1] = c;
  });
  for (int t = 0; t < T; ++t) cnt[t + 1] += cnt[t];
  parallel_for(T, [&](int t) {
    int64_t o = cnt[t];
    for (int64_t i = range_lo(n, t, T); i < range_lo(n, t + 1, T); ++i) {
      if (!h_passes(q, i)) continue;
      for (int j = 0; j < nkeep; ++j) {
        const lms_col& c = in->cols[keep[j]];
        const size_t w = (c.dtype == LMS_I32 || c.dtype == LMS_F32) ? 4 : 8;
        std::memcpy((char*)out->cols[j].data + o * w, (const char*)c.data + i * w, w);
      }
      for (int j = 0; j < nproj; ++j) {
        const int64_t v = h_proj(q, j, i);
        if (out->cols[nkeep + j].dtype == LMS_I32) ((int32_t*)out->cols[nkeep + j].data)[o] = (int32_t)v;
        else ((int64_t*)out->cols[nkeep + j].data)[o] = v;
      }
      ++o;
    }
  });
  *count = cnt[T];
  return LMS_OK;
}

extern "C" int lms_cpu_window_agg(const lms_batch* in, const lms_pred* preds, int32_t npred, const lms_proj* projs,
                                  int32_t nproj, int32_t key_col, const lms_window* w, const lms_agg* aggs,
                                  int32_t nagg, const lms_groups* out, int64_t* count, int32_t nthreads) {
  Query dummy;
  int rc = build_query(in, preds, npred, projs, nproj, &dummy);
  if (rc) return rc;
  if (!w || key_col < 0 || key_col >= in->ncols || w->ts_col < 0 || w->ts_col >= in->ncols)
    return set_error(LMS_EINVAL, "bad key/window arguments");
  if (w->len <= 0 || w->slide < 0 || w->slide > w->len) return set_error(LMS_EINVAL, "bad window length/slide");
  if (nagg < 0 || nagg > kMaxAggs || (nagg > 0 && !aggs) || !out || !count)
    return set_error(LMS_EINVAL, "bad aggregates/output");
  const int next = in->ncols + nproj;
  for (int k = 0; k < nagg; ++k)
    if (aggs[k].fn < LMS_COUNT || aggs[k].fn > LMS_AVG || (aggs[k].fn != LMS_COUNT && (aggs[k].col < 0 || aggs[k].col >= next)))
      return set_error(LMS_EINVAL, "bad aggregate %d", k);
  const int T = std::max(1, nthreads);
  const int64_t n = in->nrows;
  const int64_t S = w->slide ? w->slide : w->len;
  int64_t P = w->len, b = S;  // pane = gcd(len, slide)
  while (b) {
    const int64_t t = P % b;
    P = b;
    b = t;
  }
  const int64_t R = S / P, W = w->len / P;
  HostQuery q{in, preds, npred, projs, nproj};
  struct Row {
    int64_t key, pane;
    uint64_t v[kMaxAggs];
  };
  // 1. route passing rows to key-hash partitions
  std::vector<std::vector<std::vector<Row>>> buf(T, std::vector<std::vector<Row>>(T));
  parallel_for(T, [&](int t) {
    for (int64_t i = range_lo(n, t, T); i < range_lo(n, t + 1, T); ++i) {
      if (!h_passes(q, i)) continue;
      Row r;
      r.key = h_i64(in->cols[key_col], i);
      r.pane = floor_div(h_i64(in->cols[w->ts_col], i) - w->origin, P);
      for (int k = 0; k < nagg; ++k) {
        if (aggs[k].fn == LMS_COUNT) r.v[k] = 0;
        else if (aggs[k].fn == LMS_AVG) {
          const double d = h_ext_f64(q, aggs[k].col, i);
          std::memcpy(&r.v[k], &d, 8);
        } else {
          r.v[k] = (uint64_t)h_ext_i64(q, aggs[k].col, i);
        }
      }
      buf[t][fmix64((uint64_t)r.key) % (uint64_t)T].push_back(r);
    }
  });
  // 2. aggregate each partition, compose its windows
  struct OutRow {
    int64_t key, ws;
    uint64_t cnt;
    uint64_t v[kMaxAggs];
  };
  std::vector<std::vector<OutRow>> outs(T);
  parallel_for(T, [&](int p) {
    std::unordered_map<PaneKey, Acc, PaneKeyHash> groups;
    for (int t = 0; t < T; ++t) {
      for (const Row& r : buf[t][p]) {
        auto it = groups.find(PaneKey{r.key, r.pane});
        if (it == groups.end()) {
          Acc a;
          for (int k = 0; k < nagg; ++k) a.v[k] = r.v[k];
          a.cnt = 1;
          groups.emplace(PaneKey{r.key, r.pane}, a);
          continue;
        }
        Acc& a = it->second;
        a.cnt += 1;
        for (int k = 0; k < nagg; ++k) {
          switch (aggs[k].fn) {
            case LMS_SUM: a.v[k] += r.v[k]; break;
            case LMS_MIN: a.v[k] = (int64_t)r.v[k] < (int64_t)a.v[k] ? r.v[k] : a.v[k]; break;
            case LMS_MAX: a.v[k] = (int64_t)r.v[k] > (int64_t)a.v[k] ? r.v[k] : a.v[k]; break;
            case LMS_AVG: {
              double x, y;
              std::memcpy(&x, &a.v[k], 8);
              std::memcpy(&y, &r.v[k], 8);
              x += y;
              std::memcpy(&a.v[k], &x, 8);
              break;
            }
            default: break;
          }
        }
      }
    }
    std::unordered_map<int64_t, std::vector<std::pair<int64_t, const Acc*>>> bykey;
    for (auto& kv : groups) bykey[kv.first.key].push_back({kv.first.pane, &kv.second});
    for (auto& kv : bykey) {
      auto& ps = kv.second;
      std::sort(ps.begin(), ps.end(), [](const auto& x, const auto& y) { return x.first < y.first; });
      // windows k containing pane p: floor((p - W) / R) + 1 .. floor(p / R); sweep in order
      size_t lo = 0, next = 0;
      int64_t wk = floor_div(ps[0].first - W, R) + 1;
      while (true) {
        while (next < ps.size() && floor_div(ps[next].first - W, R) + 1 <= wk) ++next;
        while (lo < next && floor_div(ps[lo].first, R) < wk) ++lo;
        if (lo >= next) {
          if (next >= ps.size()) break;
          wk = floor_div(ps[next].first - W, R) + 1;
          continue;
        }
        OutRow o;
        o.key = kv.first;
        o.ws = w->origin + wk * S;
        o.cnt = 0;
        for (int k = 0; k < nagg; ++k) {
          const int fn = aggs[k].fn;
          o.v[k] = fn == LMS_MIN ? (uint64_t)INT64_MAX : fn == LMS_MAX ? (uint64_t)INT64_MIN : 0;
        }
        for (size_t j = lo; j < next; ++j) {
          const Acc& a = *ps[j].second;
          o.cnt += a.cnt;
          for (int k = 0; k < nagg; ++k) {
            switch (aggs[k].fn) {
              case LMS_SUM: o.v[k] += a.v[k]; break;
              case LMS_MIN: o.v[k] = (int64_t)a.v[k] < (int64_t)o.v[k] ? a.v[k] : o.v[k]; break;
              case LMS_MAX: o.v[k] = (int64_t)a.v[k] > (int64_t)o.v[k] ? a.v[k] : o.v[k]; break;
              case LMS_AVG: {
                double x, y;
                std::memcpy(&x, &o.v[k], 8);
                std::memcpy(&y, &a.v[k], 8);
                x += y;
                std::memcpy(&o.v[k], &x, 8);
                break;
              }
              default: break;
            }
          }
        }
        outs[p].push_back(o);
        ++wk;
      }
    }
  });
  // 3. concatenate
  int64_t total = 0;
  for (auto& v : outs) total += (int64_t)v.size();
  int64_t o = 0;
  for (auto& v : outs) {
    for (const OutRow& r : v) {
      if (o < out->cap) {
        out->key[o] = r.key;
        out->wstart[o] = r.ws;
        for (int k = 0; k < nagg; ++k) {
          const int fn = aggs[k].fn;
          if (fn == LMS_COUNT) ((int64_t*)out->aggs[k])[o] = (int64_t)r.cnt;
          else if (fn == LMS_AVG) {
            double x;
            std::memcpy(&x, &r.v[k], 8);
            ((double*)out->aggs[k])[o] = x / (double)r.cnt;
          } else {
            ((int64_t*)out->aggs[k])[o] = (int64_t)r.v[k];
          }
        }
      }
      ++o;
    }
  }
  *count = total;
  return LMS_OK;
}

extern "C" int lms_cpu_hash_join(const lms_batch* tbl, int32_t key_col, int32_t payload_col, const lms_batch* probe,
                                 int32_t probe_key_col, uint32_t* out_probe_idx, int32_t* out_payload, int64_t cap,
                                 int64_t* count, int32_t nthreads) {
  if (!tbl || !probe || !count || key_col < 0 || key_col >= tbl->ncols || payload_col < 0 ||
      payload_col >= tbl->ncols || probe_key_col < 0 || probe_key_col >= probe->ncols)
    return set_error(LMS_EINVAL, "bad join arguments");
  if (tbl->cols[payload_col].dtype != LMS_I32) return set_error(LMS_EINVAL, "payload column must be int32");
  const int T = std::max(1, nthreads);
  const int64_t nb = tbl->nrows, np = probe->nrows;
  uint64_t cap_slots = 64;
  while (cap_slots < 2 * (uint64_t)nb) cap_slots <<= 1;
  const uint64_t mask = cap_slots - 1;
  std::vector<int64_t> skey(cap_slots);
  std::vector<int32_t> spay(cap_slots);
  std::vector<uint8_t> used(cap_slots, 0);
  const int32_t* pay = (const int32_t*)tbl->cols[payload_col].data;
  for (int64_t j = 0; j < nb; ++j) {  // build keeps build order along each chain
    const int64_t k = h_i64(tbl->cols[key_col], j);
    uint64_t s = fmix64((uint64_t)k) & mask;
    while (used[s]) s = (s + 1) & mask;
    used[s] = 1;
    skey[s] = k;
    spay[s] = pay[j];
  }
  std::vector<std::vector<std::pair<uint32_t, int32_t>>> outs(T);
  parallel_for(T, [&](int t) {
    for (int64_t i = range_lo(np, t, T); i < range_lo(np, t + 1, T); ++i) {
      const int64_t k = h_i64(probe->cols[probe_key_col], i);
      for (uint64_t s = fmix64((uint64_t)k) & mask; used[s]; s = (s + 1) & mask)
        if (skey[s] == k) outs[t].push_back({(uint32_t)i, spay[s]});
    }
  });
  int64_t o = 0;
  for (auto& v : outs)
    for (auto& pr : v) {
      if (o < cap) {
        out_probe_idx[o] = pr.first;
        out_payload[o] = pr.second;
      }
      ++o;
    }
  *count = o;
  return LMS_OK;
}
