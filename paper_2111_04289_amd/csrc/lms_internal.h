// Internal declarations shared by the HIP sources of liblms (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lms.h"

namespace lms {

constexpr int kMaxCols = 16;
constexpr int kMaxPreds = 8;
constexpr int kMaxProjs = 8;
constexpr int kMaxAggs = 8;

// Kernel-argument image of the row-level part of a query: the columns of a
// micro-batch, a conjunction of predicates and integer projections.
struct Query {
  const void* col[kMaxCols];
  int32_t dt[kMaxCols];
  int32_t ncols;
  int32_t npred;
  int32_t nproj;
  int32_t reserved;
  int32_t pcol[kMaxPreds];
  int32_t pop[kMaxPreds];
  int64_t pival[kMaxPreds];
  double pfval[kMaxPreds];
  int32_t prsrc[kMaxProjs];
  int64_t prmul[kMaxProjs];
  int64_t pradd[kMaxProjs];
  int64_t nrows;
};

// p, which points to global memory, typed as a global pointer: accesses
// through a pointer the compiler cannot place (one read from LDS, say) are
// otherwise flat instructions, which also count against the LDS wait counter.
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gptr(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

__device__ __forceinline__ int64_t load_i64(const void* p, int dt, int64_t i) {
  return dt == LMS_I32 ? (int64_t)gptr((const int32_t*)p)[i] : gptr((const int64_t*)p)[i];
}

__device__ __forceinline__ double load_f64(const void* p, int dt, int64_t i) {
  switch (dt) {
    case LMS_I32: return (double)gptr((const int32_t*)p)[i];
    case LMS_I64: return (double)gptr((const int64_t*)p)[i];
    case LMS_F32: return (double)gptr((const float*)p)[i];
    default: return gptr((const double*)p)[i];
  }
}

template <class T>
__device__ __forceinline__ bool compare(T v, int op, T c) {
  switch (op) {
    case LMS_LT: return v < c;
    case LMS_LE: return v <= c;
    case LMS_GT: return v > c;
    case LMS_GE: return v >= c;
    case LMS_EQ: return v == c;
    default: return v != c;
  }
}

__device__ __forceinline__ bool is_int_dtype(int dt) { return dt == LMS_I32 || dt == LMS_I64; }

// Conjunction of the predicates on row i.
__device__ __forceinline__ bool row_passes(const Query& q, int64_t i) {
  bool ok = true;
  for (int k = 0; k < q.npred; ++k) {
    const int c = q.pcol[k];
    const int dt = q.dt[c];
    if (is_int_dtype(dt)) ok = ok && compare<int64_t>(load_i64(q.col[c], dt, i), q.pop[k], q.pival[k]);
    else ok = ok && compare<double>(load_f64(q.col[c], dt, i), q.pop[k], q.pfval[k]);
  }
  return ok;
}

// Rows idx[u] (where ld[u]; 0 elsewhere) of a column, U at a time.  Every
// lane issues all U loads unconditionally, a row that is not needed reading
// row `safe` (any valid row: the same line for all of them) instead, and only
// then converts: a load under a per-row branch gets its conversion or
// comparison moved into the branch, which makes the wave wait for each load
// before issuing the next one.
template <int U>
__device__ __forceinline__ void load_i64_rows(const void* p, int dt, const int64_t (&idx)[U], const bool (&ld)[U],
                                              int64_t safe, int64_t (&v)[U]) {
  if (dt == LMS_I32) {
    int32_t x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) x[u] = gptr((const int32_t*)p)[ld[u] ? idx[u] : safe];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = ld[u] ? (int64_t)x[u] : 0;
  } else {
    int64_t x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) x[u] = gptr((const int64_t*)p)[ld[u] ? idx[u] : safe];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = ld[u] ? x[u] : 0;
  }
}

template <int U>
__device__ __forceinline__ void load_f64_rows(const void* p, int dt, const int64_t (&idx)[U], const bool (&ld)[U],
                                              int64_t safe, double (&v)[U]) {
  switch (dt) {
    case LMS_F32: {
      float x[U];
#pragma unroll
      for (int u = 0; u < U; ++u) x[u] = gptr((const float*)p)[ld[u] ? idx[u] : safe];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = ld[u] ? (double)x[u] : 0.0;
      break;
    }
    case LMS_F64: {
      double x[U];
#pragma unroll
      for (int u = 0; u < U; ++u) x[u] = gptr((const double*)p)[ld[u] ? idx[u] : safe];
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = ld[u] ? x[u] : 0.0;
      break;
    }
    default: {
      int64_t x[U];
      load_i64_rows<U>(p, dt, idx, ld, safe, x);
#pragma unroll
      for (int u = 0; u < U; ++u) v[u] = (double)x[u];
    }
  }
}

// Predicates of U rows at once (rows idx[u] with valid[u]): for each predicate
// the U loads are issued together, so the rows' memory latencies overlap.
// Rows outside the range (ok[u] false on entry) read row `safe` (any valid row).
template <int U>
__device__ __forceinline__ void rows_pass(const Query& q, const int64_t (&idx)[U], bool (&ok)[U], int64_t safe) {
  for (int k = 0; k < q.npred; ++k) {
    const int c = q.pcol[k];
    const int dt = q.dt[c];
    const void* col = q.col[c];
    if (is_int_dtype(dt)) {
      int64_t v[U];
      load_i64_rows<U>(col, dt, idx, ok, safe, v);
#pragma unroll
      for (int u = 0; u < U; ++u) ok[u] = ok[u] && compare<int64_t>(v[u], q.pop[k], q.pival[k]);
    } else {
      double v[U];
      load_f64_rows<U>(col, dt, idx, ok, safe, v);
#pragma unroll
      for (int u = 0; u < U; ++u) ok[u] = ok[u] && compare<double>(v[u], q.pop[k], q.pfval[k]);
    }
  }
}

// ---- row quads ------------------------------------------------------------
// A lane takes four consecutive rows r0 .. r0 + 3 (r0 a multiple of 4) and
// loads them with one 16-byte load of a 4-byte column (two of an 8-byte one),
// where the column starts on a 16-byte boundary: a wave's load then covers 1-2
// KB instead of 256-512 B (a plain 4-byte column scan measured 6 TB/s against
// 3.2 TB/s with one row per lane at the same bytes in flight).

__device__ __forceinline__ bool wide_dtype(int dt) { return dt == LMS_I64 || dt == LMS_F64; }

// Raw 64-bit bits of U quads starting at rows r0[u].  The column width is a
// template parameter, so a caller branches on it once around the loads and
// their uses: a width branch joining between a load and its first use would
// make the wave wait for each load before issuing the next.
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
typedef uint64_t u64x2_t __attribute__((ext_vector_type(2)));

template <bool kWide, int U>
__device__ __forceinline__ void load_quads(const void* col, const int64_t (&r0)[U], uint64_t (&v)[U][4]) {
  if constexpr (kWide) {
    u64x2_t x[U], y[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t* q = (const uint64_t*)col + r0[u];
      x[u] = *gptr((const u64x2_t*)q);
      y[u] = *gptr((const u64x2_t*)(q + 2));
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      v[u][0] = x[u].x;
      v[u][1] = x[u].y;
      v[u][2] = y[u].x;
      v[u][3] = y[u].y;
    }
  } else {
    u32x4_t x[U];
#pragma unroll
    for (int u = 0; u < U; ++u) x[u] = *gptr((const u32x4_t*)((const uint32_t*)col + r0[u]));
#pragma unroll
    for (int u = 0; u < U; ++u) {
      v[u][0] = x[u].x;
      v[u][1] = x[u].y;
      v[u][2] = x[u].z;
      v[u][3] = x[u].w;
    }
  }
}

// One predicate on a value's raw bits (the comparisons of rows_pass).
__device__ __forceinline__ bool pred_bits(uint64_t b, int dt, int op, int64_t iv, double fv) {
  switch (dt) {
    case LMS_I32: return compare<int64_t>((int64_t)(int32_t)(uint32_t)b, op, iv);
    case LMS_I64: return compare<int64_t>((int64_t)b, op, iv);
    case LMS_F32: return compare<double>((double)__uint_as_float((uint32_t)b), op, fv);
    default: return compare<double>(__longlong_as_double((long long)b), op, fv);
  }
}

template <bool kWide, int U>
__device__ __forceinline__ void pred_quads(const Query& q, int k, const int64_t (&r0)[U], uint32_t (&m)[U]) {
  const int c = q.pcol[k];
  const int dt = q.dt[c], op = q.pop[k];
  const int64_t iv = q.pival[k];
  const double fv = q.pfval[k];
  uint64_t v[U][4];
  load_quads<kWide, U>(q.col[c], r0, v);
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (!pred_bits(v[u][e], dt, op, iv, fv)) m[u] &= ~(1u << e);
}

// Pass masks of U quads (bit e: row r0[u] + e), all rows in range.
template <int U>
__device__ __forceinline__ void quads_pass(const Query& q, const int64_t (&r0)[U], uint32_t (&m)[U]) {
#pragma unroll
  for (int u = 0; u < U; ++u) m[u] = 0xF;
  for (int k = 0; k < q.npred; ++k) {
    if (wide_dtype(q.dt[q.pcol[k]])) pred_quads<true, U>(q, k, r0, m);
    else pred_quads<false, U>(q, k, r0, m);
  }
}

// Whether every predicate column starts on a 16-byte boundary.
__host__ __forceinline__ bool preds_aligned(const Query& q) {
  bool ok = true;
  for (int k = 0; k < q.npred; ++k) ok = ok && ((uintptr_t)q.col[q.pcol[k]] & 15) == 0;
  return ok;
}

// Projection j of row i, wrapped to the source column's width.
__device__ __forceinline__ int64_t project(const Query& q, int j, int64_t i) {
  const int s = q.prsrc[j];
  const uint64_t raw = (uint64_t)load_i64(q.col[s], q.dt[s], i) * (uint64_t)q.prmul[j] + (uint64_t)q.pradd[j];
  return q.dt[s] == LMS_I32 ? (int64_t)(int32_t)(uint32_t)raw : (int64_t)raw;
}

// Extended columns: input columns followed by projections.
__device__ __forceinline__ int64_t ext_i64(const Query& q, int c, int64_t i) {
  return c < q.ncols ? load_i64(q.col[c], q.dt[c], i) : project(q, c - q.ncols, i);
}
__device__ __forceinline__ double ext_f64(const Query& q, int c, int64_t i) {
  return c < q.ncols ? load_f64(q.col[c], q.dt[c], i) : (double)project(q, c - q.ncols, i);
}

// ext_i64 of rows idx[u] (where ld[u]), U at a time (see load_i64_rows).
template <int U>
__device__ __forceinline__ void ext_i64_rows(const Query& q, int c, const int64_t (&idx)[U], const bool (&ld)[U],
                                             int64_t safe, int64_t (&v)[U]) {
  if (c < q.ncols) {
    load_i64_rows<U>(q.col[c], q.dt[c], idx, ld, safe, v);
    return;
  }
  const int j = c - q.ncols;
  const int s = q.prsrc[j];
  load_i64_rows<U>(q.col[s], q.dt[s], idx, ld, safe, v);
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const uint64_t raw = (uint64_t)v[u] * (uint64_t)q.prmul[j] + (uint64_t)q.pradd[j];
    v[u] = q.dt[s] == LMS_I32 ? (int64_t)(int32_t)(uint32_t)raw : (int64_t)raw;
  }
}

// MurmurHash3 64-bit finaliser (Appleby), a bijective avalanche mixer.
__host__ __device__ __forceinline__ uint64_t fmix64(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdull;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ull;
  k ^= k >> 33;
  return k;
}

__host__ __device__ __forceinline__ int64_t floor_div(int64_t a, int64_t b) {
  int64_t q = a / b;
  if ((a % b) != 0 && a < 0) q -= 1;
  return q;
}

// ---- block-wide helpers (blockDim.x = TPB, a multiple of 64) --------------

// Exclusive prefix sum of `v` over the block; `scratch` holds >= TPB/64 + 1
// words of LDS.  Returns the exclusive prefix; *total receives the block sum.
template <int TPB>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* scratch, uint32_t* total) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) scratch[wave] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int w = 0; w < TPB / 64; ++w) {
      uint32_t t = scratch[w];
      scratch[w] = run;
      run += t;
    }
    scratch[TPB / 64] = run;
  }
  __syncthreads();
  uint32_t res = scratch[wave] + x - v;
  *total = scratch[TPB / 64];
  __syncthreads();
  return res;
}

template <int TPB>
__device__ __forceinline__ uint32_t block_sum(uint32_t v, uint32_t* scratch) {
  uint32_t total;
  block_excl_scan<TPB>(v, scratch, &total);
  return total;
}

// In-place exclusive scan of arr[0..n) in LDS; returns the total.
template <int TPB>
__device__ __forceinline__ uint32_t block_scan_array(uint32_t* arr, int n, uint32_t* scratch) {
  const int per = (n + TPB - 1) / TPB;
  const int lo = threadIdx.x * per;
  const int hi = min(n, lo + per);
  uint32_t s = 0;
  for (int i = lo; i < hi; ++i) s += arr[i];
  uint32_t total;
  uint32_t run = block_excl_scan<TPB>(s, scratch, &total);
  for (int i = lo; i < hi; ++i) {
    uint32_t t = arr[i];
    arr[i] = run;
    run += t;
  }
  __syncthreads();
  return total;
}

// Single-workgroup exclusive scan of n int64 tile counts (TPB threads, each
// scanning a contiguous run); writes off[0..n) and, from thread 0, *total.
// The per-thread sums are scanned with wave shuffles and one wave over the
// wave totals, so no thread walks all TPB sums.
template <int TPB>
__device__ void tile_offsets(const int64_t* cnt, int64_t* off, int n, int64_t* total) {
  static_assert(TPB % 64 == 0 && TPB / 64 <= 64, "one wave scans the wave totals");
  __shared__ int64_t wsum[TPB / 64 + 1];
  const int per = (n + TPB - 1) / TPB;
  const int lo = threadIdx.x * per;
  const int hi = min(n, lo + per);
  constexpr int kHeld = 16;  // the first counts of the run are loaded together and kept
  int64_t held[kHeld];
  int64_t s = 0;
#pragma unroll
  for (int j = 0; j < kHeld; ++j) {
    held[j] = lo + j < hi ? cnt[lo + j] : 0;
    s += held[j];
  }
  for (int i = lo + kHeld; i < hi; ++i) s += cnt[i];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int64_t x = s;  // inclusive scan over the wave
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int64_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) wsum[wave] = x;
  __syncthreads();
  if (wave == 0) {
    const int64_t v = lane < TPB / 64 ? wsum[lane] : 0;
    int64_t y = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int64_t z = __shfl_up(y, d, 64);
      if (lane >= d) y += z;
    }
    if (lane < TPB / 64) wsum[lane] = y - v;
    if (lane == TPB / 64 - 1) wsum[TPB / 64] = y;
  }
  __syncthreads();
  if (threadIdx.x == 0) *total = wsum[TPB / 64];
  int64_t run = wsum[wave] + x - s;
#pragma unroll
  for (int j = 0; j < kHeld; ++j) {
    if (lo + j < hi) off[lo + j] = run;
    run += held[j];
  }
  for (int i = lo + kHeld; i < hi; ++i) {
    const int64_t v = cnt[i];
    off[i] = run;
    run += v;
  }
}

// Records a device-side status (negative LMS_E* code) in d_count[1].
__device__ __forceinline__ void set_device_status(int64_t* d_count, int code) {
  atomicMin((long long*)&d_count[1], (long long)code);
}

// ---- host side -------------------------------------------------------------

int set_error(int code, const char* fmt, ...);

// Kernel tracing: while lms_trace_enable(1) is in effect, a TraceScope records
// a hipEvent on `st` when it is created and another when it is destroyed.
struct TraceScope {
  int slot = -1;
  hipStream_t st;
  TraceScope(const char* name, hipStream_t s);
  ~TraceScope();
};

#define LMS_LAUNCH(name, kern, grid, block, lds, st, ...)         \
  do {                                                             \
    ::lms::TraceScope lms_trace_scope_(name, st);                  \
    hipLaunchKernelGGL(kern, grid, block, lds, st, __VA_ARGS__);   \
  } while (0)
int check_hip(hipError_t e, const char* what);

// Validates and packs the row-level query; returns LMS_OK or an error code.
int build_query(const lms_batch* in, const lms_pred* preds, int32_t npred, const lms_proj* projs, int32_t nproj,
                Query* q);

__host__ __device__ inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Bump allocator over a caller workspace (256-byte aligned slices).
struct WsCarver {
  char* base;
  size_t off = 0;
  explicit WsCarver(void* b) : base((char*)b) {}
  template <class T>
  T* take(size_t count) {
    off = align_up(off, 256);
    T* p = base ? (T*)(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
  size_t size() const { return align_up(off, 256); }
};

}  // namespace lms
