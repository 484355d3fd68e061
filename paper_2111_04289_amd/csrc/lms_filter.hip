// Filtering + Projection (Table II rows "Filtering" and "Projection"): stable
// stream compaction of the rows that pass a conjunction of predicates.
//
// Three launches: per-tile counts of passing rows (a tile is one wave's
// contiguous range), one scan of the tile counts, then a write pass that ranks
// rows with wave ballots and a running count, so rows keep their input order
// without any global atomic or workgroup barrier, and both the column loads
// and the output writes are contiguous per wave.
#include <algorithm>
#include <mutex>

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
  int32_t quads;  // every column read starts on a 16-byte boundary
  int64_t* tile_cnt;
  int64_t* tile_off;
  int64_t* d_count;
};

// Tiles belong to waves: wave tile t covers rows [t * chunk, (t + 1) * chunk)
// (chunk = kWaveRows), processed in rounds of kRows sub-rounds of 64
// consecutive rows with lane l on row b0 + u * 64 + l, so every column load of
// a wave is one contiguous run and no workgroup-level step is needed.
constexpr int kWaveRows = 64 * kRows * 8;

__device__ __forceinline__ int64_t wave_tile() { return ((int64_t)blockIdx.x * kTPB + threadIdx.x) >> 6; }

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += (uint32_t)__shfl_xor((int)v, d, 64);
  return v;
}

// Quad path (see the row quads of lms_internal.h): when every column the
// filter reads starts on a 16-byte boundary, lane l takes rows b + 4l .. b +
// 4l + 3 of each 256-row quad, kQuadSteps quads per step.
constexpr int kQuadRows = 256;
constexpr int kQuadSteps = 4;  // quads per step: their loads are in flight together
constexpr int kStepRows = kQuadRows * kQuadSteps;
static_assert(kWaveRows % kStepRows == 0, "wave tiles hold whole steps");

__device__ __forceinline__ void step_quads(int64_t b0, int lane, int64_t (&r0)[kQuadSteps]) {
#pragma unroll
  for (int u = 0; u < kQuadSteps; ++u) r0[u] = b0 + u * kQuadRows + 4 * lane;
}

__global__ __launch_bounds__(kTPB) void k_fp_count(FpArgs a) {
  const int64_t t = wave_tile();
  if (t >= a.ntiles) return;
  const int64_t lo = t * a.chunk;
  const int64_t hi = min(a.q.nrows, lo + a.chunk);
  const int lane = threadIdx.x & 63;
  int64_t b0 = lo;
  uint32_t mine = 0;  // quad path: this lane's passing rows
  if (a.quads) {
    for (; b0 + kStepRows <= hi; b0 += kStepRows) {
      int64_t r0[kQuadSteps];
      step_quads(b0, lane, r0);
      uint32_t m[kQuadSteps];
      quads_pass<kQuadSteps>(a.q, r0, m);
#pragma unroll
      for (int u = 0; u < kQuadSteps; ++u) mine += (uint32_t)__popc(m[u]);
    }
  }
  uint32_t c = wave_sum(mine);
  for (; b0 < hi; b0 += 64 * kRows) {  // the rest row by row
    int64_t idx[kRows];
    bool ok[kRows];
#pragma unroll
    for (int u = 0; u < kRows; ++u) {
      idx[u] = b0 + (int64_t)u * 64 + lane;
      ok[u] = idx[u] < hi;
    }
    rows_pass<kRows>(a.q, idx, ok, lo);
#pragma unroll
    for (int u = 0; u < kRows; ++u) c += (uint32_t)__popcll(__ballot(ok[u]));
  }
  if (lane == 0) a.tile_cnt[t] = c;
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

// Quad path of output column j: loads the step's quads of its source column
// (a kept column, or a projection's source with the projection applied, as
// out_bits gives them) and writes the passing rows from output row r[u] on.
template <bool kWide>
__device__ __forceinline__ void write_quads(const FpArgs& a, int j, const int64_t (&r0)[kQuadSteps],
                                            const uint32_t (&m)[kQuadSteps], const int64_t (&r)[kQuadSteps]) {
  const bool kept = j < a.nkeep;
  const int p = j - a.nkeep;
  const int sc = kept ? a.keep[j] : a.q.prsrc[p];
  const int dt = a.q.dt[sc];
  uint64_t v[kQuadSteps][4];
  load_quads<kWide, kQuadSteps>(a.q.col[sc], r0, v);
  if (!kept) {
    const uint64_t mul = (uint64_t)a.q.prmul[p], add = (uint64_t)a.q.pradd[p];
#pragma unroll
    for (int u = 0; u < kQuadSteps; ++u)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t x = dt == LMS_I32 ? (int64_t)(int32_t)(uint32_t)v[u][e] : (int64_t)v[u][e];
        const uint64_t raw = (uint64_t)x * mul + add;
        v[u][e] = dt == LMS_I32 ? (uint64_t)(int64_t)(int32_t)(uint32_t)raw : raw;
      }
  }
  void* const out = a.out[j];
  const int odt = a.odt[j];
#pragma unroll
  for (int u = 0; u < kQuadSteps; ++u) {
    int64_t o = r[u];
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if ((m[u] >> e) & 1u) put_bits(out, odt, o++, v[u][e]);
  }
}

// Stable compaction, one wave per tile: a passing row's output position is the
// tile's offset, plus the passing rows of the wave's earlier sub-rounds (a
// running count), plus those of lower lanes in its sub-round's ballot.  The
// passing lanes of a sub-round write one contiguous run of each column.  No
// workgroup barrier: a wave's stores drain while it moves on.
__global__ __launch_bounds__(kTPB) void k_fp_write(FpArgs a) {
  const int64_t t = wave_tile();
  if (t >= a.ntiles) return;
  const int64_t lo = t * a.chunk;
  const int64_t hi = min(a.q.nrows, lo + a.chunk);
  const int ncol = a.nkeep + a.q.nproj;
  const int lane = threadIdx.x & 63;
  const uint64_t below = (1ull << lane) - 1;
  // a dense tile (at least one row in eight passing, so nearly every cache
  // line is needed anyway) loads every row's values without waiting on the
  // predicate; a sparse one only the passing rows'
  const bool dense = a.tile_cnt[t] * 8 >= hi - lo;
  int64_t run = a.tile_off[t];
  int64_t b0 = lo;
  if (dense && a.quads) {
    // quad path: the lane's passing rows of quad u take consecutive outputs
    // from the lanes below it (their passing rows, all four slots) on
    for (; b0 + kStepRows <= hi; b0 += kStepRows) {
      int64_t r0[kQuadSteps];
      step_quads(b0, lane, r0);
      uint32_t m[kQuadSteps];
      quads_pass<kQuadSteps>(a.q, r0, m);
      int64_t r[kQuadSteps];
#pragma unroll
      for (int u = 0; u < kQuadSteps; ++u) {
        uint32_t pre = 0, tot = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const uint64_t bm = __ballot((m[u] >> e) & 1u);
          pre += (uint32_t)__popcll(bm & below);
          tot += (uint32_t)__popcll(bm);
        }
        r[u] = run + pre;
        run += tot;
      }
      // Columns a predicate read go first, while their lines still sit in
      // L2 (measured: 6 % off this kernel when the projection reads the
      // predicate column).
      for (int pass = 0; pass < 2; ++pass) {
        for (int j = 0; j < ncol; ++j) {
          const int sc = j < a.nkeep ? a.keep[j] : a.q.prsrc[j - a.nkeep];
          bool in_pred = false;
          for (int k = 0; k < a.q.npred; ++k) in_pred = in_pred || a.q.pcol[k] == sc;
          if (in_pred != (pass == 0)) continue;
          if (wide_dtype(a.q.dt[sc])) write_quads<true>(a, j, r0, m, r);
          else write_quads<false>(a, j, r0, m, r);
        }
      }
    }
  }
  for (; b0 < hi; b0 += 64 * kRows) {  // the rest row by row
    int64_t idx[kRows];
    bool pass[kRows];
#pragma unroll
    for (int u = 0; u < kRows; ++u) {
      idx[u] = b0 + (int64_t)u * 64 + lane;
      pass[u] = idx[u] < hi;
    }
    rows_pass<kRows>(a.q, idx, pass, lo);
    int64_t r[kRows];
#pragma unroll
    for (int u = 0; u < kRows; ++u) {
      const uint64_t m = __ballot(pass[u]);
      r[u] = run + __popcll(m & below);
      run += __popcll(m);
    }
    for (int j = 0; j < ncol; ++j) {
      uint64_t v[kRows];
#pragma unroll
      for (int u = 0; u < kRows; ++u) v[u] = ((dense && idx[u] < hi) || pass[u]) ? out_bits(a, j, idx[u]) : 0;
#pragma unroll
      for (int u = 0; u < kRows; ++u)
        if (pass[u]) put_bits(a.out[j], a.odt[j], r[u], v[u]);
    }
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
  p.chunk = kWaveRows;
  while ((n + p.chunk - 1) / p.chunk > (1 << 20)) p.chunk *= 2;  // at most 2^20 wave tiles
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

namespace lms {
namespace {

// Validates the call and enqueues the three launches.  `workspace` is either
// the caller's buffer or the device address of the fixed scratch array;
// ws_bytes is its size in both cases.
int fp_run(const lms_batch* in, const lms_pred* preds, int32_t npred, const int32_t* keep, int32_t nkeep,
           const lms_proj* projs, int32_t nproj, const lms_batch* out, int64_t* d_count, void* workspace,
           size_t ws_bytes, lms_stream stream) {
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
  // the quad path needs every column it reads on a 16-byte boundary
  auto aligned = [&](int c) { return ((uintptr_t)a.q.col[c] & 15) == 0; };
  bool quads = true;
  for (int k = 0; k < a.q.npred; ++k) quads = quads && aligned(a.q.pcol[k]);
  for (int j = 0; j < nkeep; ++j) quads = quads && aligned(a.keep[j]);
  for (int j = 0; j < a.q.nproj; ++j) quads = quads && aligned(a.q.prsrc[j]);
  a.quads = quads ? 1 : 0;
  const FpPlan p = fp_plan(in->nrows);
  a.chunk = p.chunk;
  a.ntiles = p.ntiles;
  a.d_count = d_count;
  hipStream_t st = (hipStream_t)stream;
  if (in->nrows == 0) {
    LMS_LAUNCH("k_fp_empty", k_fp_empty, dim3(1), dim3(64), 0, st, a);
  } else {
    const unsigned wgs = (unsigned)((p.ntiles + kTPB / 64 - 1) / (kTPB / 64));  // one wave per tile
    LMS_LAUNCH("k_fp_count", k_fp_count, dim3(wgs), dim3(kTPB), 0, st, a);
    LMS_LAUNCH("k_fp_scan", k_fp_scan, dim3(1), dim3(kScanThreads), 0, st, a);
    LMS_LAUNCH("k_fp_write", k_fp_write, dim3(wgs), dim3(kTPB), 0, st, a);
  }
  return check_hip(hipGetLastError(), "filter_project launch");
}

// Fixed scratch of the allocation-free entry point: the tile counts and tile
// offsets of up to kScratchTiles wave tiles (1 MiB per device, held until the
// process ends).  Host code never passes `scratch` itself to a kernel (in host
// code the name is a stand-in, not a device address); it uses the address
// hipGetSymbolAddress returned for the current device.
constexpr int64_t kScratchTiles = 65536;
constexpr int64_t kScratchRows = kScratchTiles * kWaveRows;  // 2^28
__device__ __align__(256) int64_t scratch[2 * kScratchTiles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices];  // device address of `scratch`, per device

int scratch_address(void** out) {
  int dev = -1;
  int rc = check_hip(hipGetDevice(&dev), "hipGetDevice");
  if (rc) return rc;
  if (dev < 0 || dev >= kMaxDevices) return set_error(LMS_EINVAL, "device %d beyond the %d supported", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    rc = check_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (rc) return rc;
    if (!p) return set_error(LMS_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return LMS_OK;
}

}  // namespace
}  // namespace lms

extern "C" int lms_filter_project(const lms_batch* in, const lms_pred* preds, int32_t npred, const int32_t* keep,
                                  int32_t nkeep, const lms_proj* projs, int32_t nproj, const lms_batch* out,
                                  int64_t* d_count, void* workspace, size_t ws_bytes, lms_stream stream) {
  return fp_run(in, preds, npred, keep, nkeep, projs, nproj, out, d_count, workspace, ws_bytes, stream);
}

extern "C" int64_t lms_filter_project_noalloc_max_rows(void) { return kScratchRows; }

extern "C" int lms_filter_project_noalloc(const lms_batch* in, const lms_pred* preds, int32_t npred,
                                          const int32_t* keep, int32_t nkeep, const lms_proj* projs, int32_t nproj,
                                          const lms_batch* out, int64_t* d_count, lms_stream stream) {
  if (!in) return set_error(LMS_EINVAL, "input batch is NULL");
  if (in->nrows > kScratchRows)
    return set_error(LMS_EINVAL, "%lld rows exceed the %lld the fixed scratch of lms_filter_project_noalloc covers",
                     (long long)in->nrows, (long long)kScratchRows);
  void* ws = nullptr;
  int rc = scratch_address(&ws);
  if (rc) return rc;
  return fp_run(in, preds, npred, keep, nkeep, projs, nproj, out, d_count, ws, sizeof(int64_t) * 2 * kScratchTiles,
                stream);
}
