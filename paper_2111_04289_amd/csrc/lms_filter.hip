// Filtering + Projection (Table II rows "Filtering" and "Projection"): stable
// stream compaction of the rows that pass a conjunction of predicates.
//
// Three launches: per-tile counts of passing rows, one scan of the tile
// counts, then a write pass that ranks each round of rows with wave ballots
// and a block prefix, so rows keep their input order without any global
// atomic, and both the column loads and the output writes are contiguous per
// wave.
#include <algorithm>

#include "lms_internal.h"

namespace lms {
namespace {

constexpr int kTPB = 256;
constexpr int kScanThreads = 1024;
constexpr int kRows = 8;

struct FpArgs {
  Query q;
  int32_t nkeep;
  int32_t keep[kMaxCols];
  void* out[kMaxCols + kMaxProjs];
  int32_t odt[kMaxCols + kMaxProjs];
  int64_t chunk;
  int32_t ntiles;
  int64_t* tile_cnt;
  int64_t* tile_off;
  int64_t* d_count;
};

// A round is kRows sub-rounds of kTPB consecutive rows; in sub-round u lane t
// takes row b0 + u * kTPB + t, so every column load of a wave is one
// contiguous run.
__global__ __launch_bounds__(kTPB) void k_fp_count(FpArgs a) {
  __shared__ uint32_t scratch[kTPB / 64 + 1];
  const int64_t lo = (int64_t)blockIdx.x * a.chunk;
  const int64_t hi = min(a.q.nrows, lo + a.chunk);
  uint32_t c = 0;
  for (int64_t b0 = lo; b0 < hi; b0 += (int64_t)kTPB * kRows) {
    int64_t idx[kRows];
    bool ok[kRows];
#pragma unroll
    for (int u = 0; u < kRows; ++u) {
      idx[u] = b0 + (int64_t)u * kTPB + threadIdx.x;
      ok[u] = idx[u] < hi;
    }
    rows_pass<kRows>(a.q, idx, ok);
#pragma unroll
    for (int u = 0; u < kRows; ++u) c += ok[u] ? 1u : 0u;
  }
  c = block_sum<kTPB>(c, scratch);
  if (threadIdx.x == 0) a.tile_cnt[blockIdx.x] = c;
}

__global__ __launch_bounds__(kScanThreads) void k_fp_scan(FpArgs a) {
  __shared__ int64_t total;
  tile_offsets<kScanThreads>(a.tile_cnt, a.tile_off, a.ntiles, &total);
  __syncthreads();
  if (threadIdx.x == 0) {
    a.d_count[0] = total;
    a.d_count[1] = 0;
  }
}

// Value of output column j for input row i, as raw 64-bit bits.
__device__ __forceinline__ uint64_t out_bits(const FpArgs& a, int j, int64_t i) {
  if (j >= a.nkeep) return (uint64_t)project(a.q, j - a.nkeep, i);
  const int c = a.keep[j];
  switch (a.q.dt[c]) {
    case LMS_I32: return (uint64_t)(uint32_t)((const int32_t*)a.q.col[c])[i];
    case LMS_F32: return (uint64_t)__float_as_uint(((const float*)a.q.col[c])[i]);
    default: return ((const uint64_t*)a.q.col[c])[i];
  }
}

__device__ __forceinline__ void put_bits(void* col, int dt, int64_t r, uint64_t v) {
  if (dt == LMS_I32 || dt == LMS_F32) ((uint32_t*)col)[r] = (uint32_t)v;
  else ((uint64_t*)col)[r] = v;
}

// Stable compaction.  Ranks come from wave ballots: a passing row's rank is
// the passing rows of earlier (sub-round, wave) pairs -- sub-round major, as
// rows are ordered -- plus those of lower lanes in its wave's ballot.  The
// passing lanes of a wave therefore write one contiguous run of each output
// column, and every load is contiguous too; no value is staged.
__global__ __launch_bounds__(kTPB) void k_fp_write(FpArgs a) {
  constexpr int kWaves = kTPB / 64;
  __shared__ uint32_t wpre[kRows * kWaves + 1];
  const int64_t lo = (int64_t)blockIdx.x * a.chunk;
  const int64_t hi = min(a.q.nrows, lo + a.chunk);
  const int ncol = a.nkeep + a.q.nproj;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t below = (1ull << lane) - 1;
  int64_t run = a.tile_off[blockIdx.x];
  const bool dense = a.tile_cnt[blockIdx.x] * 8 >= hi - lo;
  for (int64_t b0 = lo; b0 < hi; b0 += (int64_t)kTPB * kRows) {
    int64_t idx[kRows];
    bool pass[kRows];
#pragma unroll
    for (int u = 0; u < kRows; ++u) {
      idx[u] = b0 + (int64_t)u * kTPB + threadIdx.x;
      pass[u] = idx[u] < hi;
    }
    rows_pass<kRows>(a.q, idx, pass);
    uint64_t m[kRows];
#pragma unroll
    for (int u = 0; u < kRows; ++u) {
      m[u] = __ballot(pass[u]);
      if (lane == 0) wpre[u * kWaves + wave] = (uint32_t)__popcll(m[u]);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t t = 0;
      for (int i = 0; i < kRows * kWaves; ++i) {
        const uint32_t v = wpre[i];
        wpre[i] = t;
        t += v;
      }
      wpre[kRows * kWaves] = t;
    }
    __syncthreads();
    int64_t r[kRows];
#pragma unroll
    for (int u = 0; u < kRows; ++u) r[u] = run + wpre[u * kWaves + wave] + __popcll(m[u] & below);
    // per column, the rows' values are loaded together before any is stored, so
    // the loads of a round overlap; a dense tile (at least one row in eight
    // passing, so nearly every cache line is needed anyway) loads every row
    // without waiting on the predicate, a sparse one only the passing rows
    for (int j = 0; j < ncol; ++j) {
      uint64_t v[kRows];
#pragma unroll
      for (int u = 0; u < kRows; ++u) v[u] = ((dense && idx[u] < hi) || pass[u]) ? out_bits(a, j, idx[u]) : 0;
#pragma unroll
      for (int u = 0; u < kRows; ++u)
        if (pass[u]) put_bits(a.out[j], a.odt[j], r[u], v[u]);
    }
    run += wpre[kRows * kWaves];
    __syncthreads();  // wpre is rewritten by the next round
  }
}

__global__ void k_fp_empty(FpArgs a) {
  if (threadIdx.x == 0) {
    a.d_count[0] = 0;
    a.d_count[1] = 0;
  }
}

struct FpPlan {
  int64_t chunk;
  int ntiles;
};

FpPlan fp_plan(int64_t n) {
  FpPlan p;
  p.chunk = 8192;  // measured: larger tiles serialise the rounds of a workgroup and run slower
  while ((n + p.chunk - 1) / p.chunk > 65536) p.chunk *= 2;
  p.ntiles = (int)((n + p.chunk - 1) / p.chunk);
  return p;
}

size_t fp_workspace(int64_t n, FpArgs* a, void* base) {
  const FpPlan p = fp_plan(n);
  WsCarver c(base);
  int64_t* cnt = c.take<int64_t>(std::max(1, p.ntiles));
  int64_t* off = c.take<int64_t>(std::max(1, p.ntiles));
  if (a) {
    a->tile_cnt = cnt;
    a->tile_off = off;
  }
  return c.size();
}

}  // namespace
}  // namespace lms

using namespace lms;

extern "C" size_t lms_filter_project_workspace(int64_t nrows) {
  return nrows < 0 ? 0 : fp_workspace(nrows, nullptr, nullptr);
}

extern "C" int lms_filter_project(const lms_batch* in, const lms_pred* preds, int32_t npred, const int32_t* keep,
                                  int32_t nkeep, const lms_proj* projs, int32_t nproj, const lms_batch* out,
                                  int64_t* d_count, void* workspace, size_t ws_bytes, lms_stream stream) {
  FpArgs a{};
  int rc = build_query(in, preds, npred, projs, nproj, &a.q);
  if (rc) return rc;
  if (nkeep < 0 || nkeep > kMaxCols) return set_error(LMS_EINVAL, "nkeep %d outside [0, %d]", nkeep, kMaxCols);
  if (nkeep > 0 && !keep) return set_error(LMS_EINVAL, "keep is NULL");
  if (!out || out->ncols != nkeep + nproj) return set_error(LMS_EINVAL, "output must have nkeep + nproj columns");
  if (out->ncols > 0 && !out->cols) return set_error(LMS_EINVAL, "output cols is NULL");
  if (!d_count) return set_error(LMS_EINVAL, "d_count is NULL");
  a.nkeep = nkeep;
  for (int j = 0; j < nkeep; ++j) {
    if (keep[j] < 0 || keep[j] >= in->ncols) return set_error(LMS_EINVAL, "keep[%d] = %d out of range", j, keep[j]);
    a.keep[j] = keep[j];
    if (out->cols[j].dtype != in->cols[keep[j]].dtype)
      return set_error(LMS_EINVAL, "output column %d must have the dtype of input column %d", j, keep[j]);
  }
  for (int j = 0; j < nproj; ++j)
    if (out->cols[nkeep + j].dtype != in->cols[projs[j].src].dtype)
      return set_error(LMS_EINVAL, "output column %d must have the dtype of projection %d's source", nkeep + j, j);
  for (int j = 0; j < out->ncols; ++j) {
    if (in->nrows > 0 && !out->cols[j].data) return set_error(LMS_EINVAL, "output column %d is NULL", j);
    a.out[j] = out->cols[j].data;
    a.odt[j] = out->cols[j].dtype;
  }
  const size_t need = fp_workspace(in->nrows, nullptr, nullptr);
  if (!workspace || ws_bytes < need)
    return set_error(LMS_ENOMEM, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
  fp_workspace(in->nrows, &a, workspace);
  const FpPlan p = fp_plan(in->nrows);
  a.chunk = p.chunk;
  a.ntiles = p.ntiles;
  a.d_count = d_count;
  hipStream_t st = (hipStream_t)stream;
  if (in->nrows == 0) {
    LMS_LAUNCH("k_fp_empty", k_fp_empty, dim3(1), dim3(64), 0, st, a);
  } else {
    LMS_LAUNCH("k_fp_count", k_fp_count, dim3(p.ntiles), dim3(kTPB), 0, st, a);
    LMS_LAUNCH("k_fp_scan", k_fp_scan, dim3(1), dim3(kScanThreads), 0, st, a);
    LMS_LAUNCH("k_fp_write", k_fp_write, dim3(p.ntiles), dim3(kTPB), 0, st, a);
  }
  return check_hip(hipGetLastError(), "filter_project launch");
}
