// Device-resident window state for a stream of micro-batches.
//
// A windowed group-by over a stream (Sec. II-A's window semantics applied
// across micro-batches) needs the partial aggregates of windows that are still
// open when a micro-batch ends.  The state keeps them per (key, pane) in HBM,
// where a pane is gcd(range, slide) long, so one row updates exactly one entry
// and a window is composed from its range/pane consecutive panes when emitted:
//
//   * key dictionary: open addressing over int64 keys (CAS insert); a key's
//     slot index is its id, so no second table is needed.  One extra slot
//     holds the key whose value equals the empty marker.
//   * pane ring: per key, `ring` entries indexed by pane mod ring, each tagged
//     with the pane it holds; laid out [ring][key slot] so that a sweep over
//     key slots at a fixed ring index is coalesced.
//   * accumulators per entry: count plus one 64-bit word per non-COUNT
//     aggregate (int64 SUM/MIN/MAX, FP64 sum for AVG).
//
// update: every passing row atomically adds into its (key, pane) entry.
// emit:   windows that end at or before the watermark (all remaining ones when
//         flushing), in order and each once, are composed per key and written
//         out; then the panes no later window needs are cleared.  A row whose
//         pane lies only in windows already emitted is late: it is counted and
//         dropped.
// All control state (next window, pane range seen) lives in device memory, so
// the calls are stream-ordered with no host synchronisation.
#include <algorithm>
#include <climits>

#include "lms_internal.h"

namespace lms {
namespace {

constexpr uint64_t kNoKey = 0x8000000000000000ull;
constexpr int64_t kNoPane = INT64_MIN;
constexpr int kTPB = 256;

// Device control words.
enum : int {
  kLate = 0,      // rows dropped as late
  kDropped = 1,   // rows dropped for lack of capacity
  kMinPane = 2,   // smallest pane updated so far (INT64_MAX before any row)
  kMaxPane = 3,   // largest pane updated so far (INT64_MIN before any row)
  kNextWin = 4,   // next window to emit (INT64_MIN: from the first pane seen)
  kEmitLo = 5,    // window range of the last emit
  kEmitHi = 6,
  kStatus = 7,    // LMS_ECAPACITY once a row did not fit
  kNumCtl = 8
};

struct StateArgs {
  int64_t* keys;    // kslots (+1 for the empty-marker key)
  int64_t* tags;    // ring * (kslots + 1)
  uint64_t* cnt;    // ring * (kslots + 1)
  uint64_t* acc[kMaxAggs];
  int64_t* ctl;
  int64_t kslots;   // power of two
  int64_t stride;   // kslots + 1: entries per ring index
  int32_t ring;     // power of two
  int32_t nacc;
  int32_t accfn[kMaxAggs];   // LMS_SUM / MIN / MAX / AVG
  int32_t acccol[kMaxAggs];  // extended column of accumulator s
  int64_t len, slide, origin, pane, R, W;
  int32_t ts_col, reserved;
};

}  // namespace
}  // namespace lms

struct lms_wstate {
  lms::StateArgs a;
  int32_t nagg;
  lms_agg aggs[lms::kMaxAggs];
  int32_t aggacc[lms::kMaxAggs];  // accumulator of aggregate k (-1 for COUNT)
  void* block;                    // the one allocation holding every array
};

namespace lms {
namespace {

__device__ __forceinline__ uint64_t acc_init(int fn) {
  switch (fn) {
    case LMS_MIN: return (uint64_t)INT64_MAX;
    case LMS_MAX: return (uint64_t)INT64_MIN;
    default: return 0;  // int64 0 and FP64 +0.0 share the bit pattern
  }
}

__device__ __forceinline__ void clear_entry(const StateArgs& a, int64_t e) {
  a.tags[e] = kNoPane;
  a.cnt[e] = 0;
  for (int s = 0; s < a.nacc; ++s) a.acc[s][e] = acc_init(a.accfn[s]);
}

__global__ void k_ws_zero_count(int64_t* d_count) {
  if (threadIdx.x < 2) d_count[threadIdx.x] = 0;
}

__global__ void k_ws_init(StateArgs a) {
  const int64_t total = (int64_t)a.ring * a.stride;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    clear_entry(a, i);
    if (i < a.stride) a.keys[i] = (int64_t)kNoKey;
  }
  if (blockIdx.x == 0 && threadIdx.x < kNumCtl) {
    const int64_t v[kNumCtl] = {0, 0, INT64_MAX, INT64_MIN, INT64_MIN, 0, -1, 0};
    a.ctl[threadIdx.x] = v[threadIdx.x];
  }
}

// Key slot of `key`, inserting it if absent; -1 if the dictionary is full.
__device__ __forceinline__ int64_t key_slot(const StateArgs& a, int64_t key) {
  if ((uint64_t)key == kNoKey) return a.kslots;  // the reserved extra slot
  const uint64_t mask = (uint64_t)a.kslots - 1;
  uint64_t h = fmix64((uint64_t)key) & mask;
  for (int64_t probe = 0; probe < a.kslots; ++probe) {
    const uint64_t cur = (uint64_t)a.keys[h];
    if (cur == (uint64_t)key) return (int64_t)h;
    if (cur == kNoKey) {
      const uint64_t old = atomicCAS((unsigned long long*)&a.keys[h], (unsigned long long)kNoKey,
                                     (unsigned long long)key);
      if (old == kNoKey || old == (uint64_t)key) return (int64_t)h;
    }
    h = (h + 1) & mask;
  }
  return -1;
}

__global__ __launch_bounds__(kTPB) void k_ws_update(StateArgs a, Query q, int32_t key_col) {
  const int32_t ts_col = a.ts_col;
  // panes below the first window still to emit belong only to emitted windows
  const int64_t next = a.ctl[kNextWin];
  const int64_t low = next == INT64_MIN ? INT64_MIN : next * a.R;
  int64_t qmin = INT64_MAX, qmax = INT64_MIN, late = 0, dropped = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < q.nrows; i += (int64_t)gridDim.x * blockDim.x) {
    if (!row_passes(q, i)) continue;
    const int64_t ts = load_i64(q.col[ts_col], q.dt[ts_col], i);
    const int64_t pane = floor_div(ts - a.origin, a.pane);
    if (pane < low) {
      ++late;
      continue;
    }
    const int64_t slot = key_slot(a, load_i64(q.col[key_col], q.dt[key_col], i));
    if (slot < 0) {
      ++dropped;
      continue;
    }
    const int64_t e = (pane & (a.ring - 1)) * a.stride + slot;
    const int64_t old = (int64_t)atomicCAS((unsigned long long*)&a.tags[e], (unsigned long long)kNoPane,
                                           (unsigned long long)pane);
    if (old != kNoPane && old != pane) {  // the ring entry still holds another live pane
      ++dropped;
      continue;
    }
    qmin = min(qmin, pane);
    qmax = max(qmax, pane);
    atomicAdd((unsigned long long*)&a.cnt[e], 1ull);
    for (int s = 0; s < a.nacc; ++s) {
      const int c = a.acccol[s];
      switch (a.accfn[s]) {
        case LMS_SUM: atomicAdd((unsigned long long*)&a.acc[s][e], (unsigned long long)ext_i64(q, c, i)); break;
        case LMS_MIN: atomicMin((long long*)&a.acc[s][e], (long long)ext_i64(q, c, i)); break;
        case LMS_MAX: atomicMax((long long*)&a.acc[s][e], (long long)ext_i64(q, c, i)); break;
        default: atomicAdd((double*)&a.acc[s][e], ext_f64(q, c, i)); break;
      }
    }
  }
  // one set of control updates per wave
  for (int d = 32; d >= 1; d >>= 1) {
    qmin = min(qmin, (int64_t)__shfl_xor((long long)qmin, d, 64));
    qmax = max(qmax, (int64_t)__shfl_xor((long long)qmax, d, 64));
    late += (int64_t)__shfl_xor((long long)late, d, 64);
    dropped += (int64_t)__shfl_xor((long long)dropped, d, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    if (qmin != INT64_MAX) atomicMin((long long*)&a.ctl[kMinPane], (long long)qmin);
    if (qmax != INT64_MIN) atomicMax((long long*)&a.ctl[kMaxPane], (long long)qmax);
    if (late) atomicAdd((unsigned long long*)&a.ctl[kLate], (unsigned long long)late);
    if (dropped) {
      atomicAdd((unsigned long long*)&a.ctl[kDropped], (unsigned long long)dropped);
      atomicMin((long long*)&a.ctl[kStatus], (long long)LMS_ECAPACITY);
    }
  }
}

// Window range [lo, hi] an emit call covers (empty when hi < lo).
__device__ __forceinline__ void emit_range(const StateArgs& a, int64_t watermark, int flush, int64_t max_windows,
                                           int64_t* lo, int64_t* hi) {
  const int64_t qmin = a.ctl[kMinPane], qmax = a.ctl[kMaxPane];
  *lo = 0;
  *hi = -1;
  if (qmax == INT64_MIN) return;  // no data yet
  int64_t l = a.ctl[kNextWin];
  if (l == INT64_MIN) l = floor_div(qmin - a.W, a.R) + 1;  // first window holding the first pane
  int64_t h = floor_div(qmax, a.R);                        // last window holding data
  if (!flush) h = min(h, floor_div(watermark - a.origin - a.len, a.slide));
  h = min(h, l + max_windows - 1);
  *lo = l;
  *hi = h;
}

struct EmitOut {
  int64_t* key;
  int64_t* wstart;
  void* agg[kMaxAggs];
  int32_t afn[kMaxAggs];
  int32_t aacc[kMaxAggs];
  int32_t nagg;
  int64_t cap;
  int64_t* d_count;
};

__global__ __launch_bounds__(kTPB) void k_ws_emit(StateArgs a, EmitOut o, int64_t watermark, int32_t flush,
                                                  int64_t max_windows) {
  int64_t wlo, whi;
  emit_range(a, watermark, flush, max_windows, &wlo, &whi);
  if (whi < wlo) return;
  const int lane = threadIdx.x & 63;
  // every lane of a wave runs the same number of rounds so the ballots line up
  const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
  const int64_t rounds = (a.stride + nthreads - 1) / nthreads;
  for (int64_t r = 0; r < rounds; ++r) {
    const int64_t slot = r * nthreads + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const bool live = slot < a.stride && (uint64_t)a.keys[slot] != kNoKey;
    const int64_t key = slot == a.kslots ? (int64_t)kNoKey : (live ? a.keys[slot] : 0);
    bool live_key = live;
    if (slot == a.kslots) {  // the empty-marker key is present iff one of its entries is in use
      live_key = false;
      for (int ri = 0; ri < a.ring; ++ri) live_key |= a.tags[(int64_t)ri * a.stride + slot] != kNoPane;
    }
    for (int64_t w = wlo; w <= whi; ++w) {
      uint64_t cnt = 0;
      uint64_t acc[kMaxAggs];
      for (int s = 0; s < kMaxAggs; ++s) acc[s] = s < a.nacc ? acc_init(a.accfn[s]) : 0;
      if (live_key) {
        for (int64_t p = w * a.R; p < w * a.R + a.W; ++p) {
          const int64_t e = (p & (a.ring - 1)) * a.stride + slot;
          if (a.tags[e] != p) continue;
          cnt += a.cnt[e];
          for (int s = 0; s < a.nacc; ++s) {
            const uint64_t v = a.acc[s][e];
            switch (a.accfn[s]) {
              case LMS_SUM: acc[s] += v; break;
              case LMS_MIN: acc[s] = (uint64_t)min((int64_t)acc[s], (int64_t)v); break;
              case LMS_MAX: acc[s] = (uint64_t)max((int64_t)acc[s], (int64_t)v); break;
              default: acc[s] = __double_as_longlong(__longlong_as_double(acc[s]) + __longlong_as_double(v)); break;
            }
          }
        }
      }
      const bool out = cnt > 0;
      const uint64_t ball = __ballot(out);
      const int nout = __popcll(ball);
      if (nout == 0) continue;
      int64_t base = 0;
      if (lane == 0) base = (int64_t)atomicAdd((unsigned long long*)&o.d_count[0], (unsigned long long)nout);
      base = (int64_t)__shfl((long long)base, 0, 64);
      if (!out) continue;
      const int64_t pos = base + __popcll(ball & ((1ull << lane) - 1));
      if (pos >= o.cap) {
        set_device_status(o.d_count, LMS_ECAPACITY);
        continue;
      }
      o.key[pos] = key;
      o.wstart[pos] = a.origin + w * a.slide;
      for (int k = 0; k < o.nagg; ++k) {
        const int s = o.aacc[k];
        switch (o.afn[k]) {
          case LMS_COUNT: ((int64_t*)o.agg[k])[pos] = (int64_t)cnt; break;
          case LMS_AVG: ((double*)o.agg[k])[pos] = __longlong_as_double(acc[s]) / (double)cnt; break;
          default: ((int64_t*)o.agg[k])[pos] = (int64_t)acc[s]; break;
        }
      }
    }
  }
}

// After an emit: record the range and move the next window past it.
__global__ void k_ws_advance(StateArgs a, int64_t watermark, int32_t flush, int64_t max_windows) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int64_t wlo, whi;
  emit_range(a, watermark, flush, max_windows, &wlo, &whi);
  a.ctl[kEmitLo] = wlo;
  a.ctl[kEmitHi] = whi;
  if (whi >= wlo) a.ctl[kNextWin] = whi + 1;
}

// Clears the ring entries of panes [p0, p1): no window from the next one on
// needs them.  p0/p1 come from the range the preceding advance recorded.
__global__ __launch_bounds__(kTPB) void k_ws_evict(StateArgs a) {
  const int64_t wlo = a.ctl[kEmitLo], whi = a.ctl[kEmitHi];
  if (whi < wlo) return;
  const int64_t p0 = min(wlo * a.R, a.ctl[kMinPane]);
  const int64_t p1 = (whi + 1) * a.R;
  const bool all = p1 - p0 >= a.ring;
  const int64_t nr = all ? a.ring : p1 - p0;
  const int64_t total = nr * a.stride;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = i / a.stride;
    const int64_t slot = i - j * a.stride;
    const int64_t ri = all ? j : ((p0 + j) & (a.ring - 1));
    const int64_t e = ri * a.stride + slot;
    const int64_t t = a.tags[e];
    if (t != kNoPane && t < p1) clear_entry(a, e);
  }
}

int grid_for(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + kTPB - 1) / kTPB, 4096)); }

int64_t next_pow2_i64(int64_t x) {
  int64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

int64_t gcd_i64(int64_t x, int64_t y) {
  while (y) {
    const int64_t t = x % y;
    x = y;
    y = t;
  }
  return x;
}

size_t state_bytes(int64_t kslots, int32_t ring, int nacc) {
  const size_t stride = (size_t)kslots + 1;
  return align_up(stride * 8, 256) + (size_t)(2 + nacc) * align_up((size_t)ring * stride * 8, 256) +
         align_up(kNumCtl * 8, 256);
}

}  // namespace
}  // namespace lms

using namespace lms;

extern "C" size_t lms_wstate_bytes(int64_t max_keys, int32_t ring_panes, int32_t nagg) {
  if (max_keys <= 0 || ring_panes <= 0 || nagg < 0 || nagg > kMaxAggs) return 0;
  return state_bytes(next_pow2_i64(2 * max_keys), (int32_t)next_pow2_i64(ring_panes), nagg);
}

extern "C" int lms_wstate_create(const lms_window* w, const lms_agg* aggs, int32_t nagg, int64_t max_keys,
                                 int32_t ring_panes, lms_wstate** out, lms_stream stream) {
  if (!out) return set_error(LMS_EINVAL, "out is NULL");
  *out = nullptr;
  if (!w || w->len <= 0 || w->slide < 0 || w->slide > w->len)
    return set_error(LMS_EINVAL, "window needs len > 0 and 0 <= slide <= len");
  if (nagg < 0 || nagg > kMaxAggs || (nagg > 0 && !aggs)) return set_error(LMS_EINVAL, "bad aggregates");
  if (max_keys <= 0 || max_keys > (1ll << 40)) return set_error(LMS_EINVAL, "max_keys out of range");
  const int64_t slide = w->slide == 0 ? w->len : w->slide;
  const int64_t pane = gcd_i64(w->len, slide);
  const int32_t ring = (int32_t)next_pow2_i64(std::max<int64_t>(ring_panes, w->len / pane + slide / pane));
  if (ring > (1 << 20)) return set_error(LMS_EINVAL, "ring of %d panes is too large", ring);
  lms_wstate* st = new lms_wstate{};
  StateArgs& a = st->a;
  a.kslots = next_pow2_i64(2 * max_keys);  // load factor <= 0.5
  a.stride = a.kslots + 1;
  a.ring = ring;
  a.ts_col = w->ts_col;
  a.len = w->len;
  a.slide = slide;
  a.origin = w->origin;
  a.pane = pane;
  a.R = slide / pane;
  a.W = w->len / pane;
  st->nagg = nagg;
  for (int k = 0; k < nagg; ++k) {
    st->aggs[k] = aggs[k];
    if (aggs[k].fn == LMS_COUNT) {
      st->aggacc[k] = -1;
      continue;
    }
    if (aggs[k].fn < LMS_COUNT || aggs[k].fn > LMS_AVG) {
      delete st;
      return set_error(LMS_EINVAL, "aggregate %d has bad function %d", k, aggs[k].fn);
    }
    st->aggacc[k] = a.nacc;
    a.accfn[a.nacc] = aggs[k].fn;
    a.acccol[a.nacc] = aggs[k].col;
    ++a.nacc;
  }
  const size_t bytes = state_bytes(a.kslots, ring, a.nacc);
  int rc = check_hip(hipMalloc(&st->block, bytes), "hipMalloc window state");
  if (rc) {
    delete st;
    return rc;
  }
  WsCarver c(st->block);
  a.keys = c.take<int64_t>(a.stride);
  a.tags = c.take<int64_t>((size_t)ring * a.stride);
  a.cnt = c.take<uint64_t>((size_t)ring * a.stride);
  for (int s = 0; s < a.nacc; ++s) a.acc[s] = c.take<uint64_t>((size_t)ring * a.stride);
  a.ctl = c.take<int64_t>(kNumCtl);
  LMS_LAUNCH("k_ws_init", k_ws_init, dim3(grid_for((int64_t)ring * a.stride)), dim3(kTPB), 0, (hipStream_t)stream, a);
  rc = check_hip(hipGetLastError(), "window state init");
  if (rc) {
    (void)hipFree(st->block);
    delete st;
    return rc;
  }
  *out = st;
  return LMS_OK;
}

extern "C" int lms_wstate_update(lms_wstate* st, const lms_batch* in, const lms_pred* preds, int32_t npred,
                                 const lms_proj* projs, int32_t nproj, int32_t key_col, lms_stream stream) {
  if (!st) return set_error(LMS_EINVAL, "state is NULL");
  Query q;
  int rc = build_query(in, preds, npred, projs, nproj, &q);
  if (rc) return rc;
  if (key_col < 0 || key_col >= in->ncols || !(in->cols[key_col].dtype == LMS_I32 || in->cols[key_col].dtype == LMS_I64))
    return set_error(LMS_EINVAL, "key column must be an int32/int64 input column");
  const int32_t ts_col = st->a.ts_col;
  if (ts_col < 0 || ts_col >= in->ncols || in->cols[ts_col].dtype != LMS_I64)
    return set_error(LMS_EINVAL, "timestamp column must be an int64 input column");
  const StateArgs& a = st->a;
  for (int s = 0; s < a.nacc; ++s) {
    const int c = a.acccol[s];
    if (c < 0 || c >= in->ncols + nproj) return set_error(LMS_EINVAL, "aggregate column %d out of range", c);
    const int dt = c < in->ncols ? in->cols[c].dtype : in->cols[projs[c - in->ncols].src].dtype;
    if (a.accfn[s] != LMS_AVG && !(dt == LMS_I32 || dt == LMS_I64))
      return set_error(LMS_EINVAL, "SUM/MIN/MAX need an integer column (column %d)", c);
  }
  if (in->nrows == 0) return LMS_OK;
  LMS_LAUNCH("k_ws_update", k_ws_update, dim3(grid_for(in->nrows)), dim3(kTPB), 0, (hipStream_t)stream, a, q, key_col);
  return check_hip(hipGetLastError(), "window state update");
}

extern "C" int lms_wstate_emit(lms_wstate* st, int64_t watermark, int32_t flush, int32_t max_windows,
                               const lms_groups* out, int64_t* d_count, lms_stream stream) {
  if (!st || !out || !d_count) return set_error(LMS_EINVAL, "NULL argument");
  if (max_windows <= 0) return set_error(LMS_EINVAL, "max_windows must be positive");
  if (out->cap < 0 || (out->cap > 0 && (!out->key || !out->wstart))) return set_error(LMS_EINVAL, "bad output");
  if (st->nagg > 0 && !out->aggs) return set_error(LMS_EINVAL, "output aggs is NULL");
  EmitOut o{};
  o.key = out->key;
  o.wstart = out->wstart;
  o.nagg = st->nagg;
  for (int k = 0; k < st->nagg; ++k) {
    if (out->cap > 0 && !out->aggs[k]) return set_error(LMS_EINVAL, "output aggregate %d is NULL", k);
    o.agg[k] = out->aggs[k];
    o.afn[k] = st->aggs[k].fn;
    o.aacc[k] = st->aggacc[k];
  }
  o.cap = out->cap;
  o.d_count = d_count;
  hipStream_t s = (hipStream_t)stream;
  const StateArgs& a = st->a;
  LMS_LAUNCH("k_ws_zero", k_ws_zero_count, dim3(1), dim3(64), 0, s, d_count);
  LMS_LAUNCH("k_ws_emit", k_ws_emit, dim3(grid_for(a.stride)), dim3(kTPB), 0, s, a, o, watermark, flush,
             (int64_t)max_windows);
  LMS_LAUNCH("k_ws_advance", k_ws_advance, dim3(1), dim3(64), 0, s, a, watermark, flush, (int64_t)max_windows);
  LMS_LAUNCH("k_ws_evict", k_ws_evict, dim3(grid_for(std::min<int64_t>(a.ring, 64) * a.stride)), dim3(kTPB), 0, s, a);
  return check_hip(hipGetLastError(), "window state emit");
}

extern "C" int lms_wstate_info(lms_wstate* st, int64_t* d_info, lms_stream stream) {
  if (!st || !d_info) return set_error(LMS_EINVAL, "NULL argument");
  return check_hip(hipMemcpyAsync(d_info, st->a.ctl, kNumCtl * sizeof(int64_t), hipMemcpyDeviceToDevice,
                                  (hipStream_t)stream),
                   "window state info");
}

extern "C" void lms_wstate_free(lms_wstate* st) {
  if (!st) return;
  (void)hipFree(st->block);
  delete st;
}
