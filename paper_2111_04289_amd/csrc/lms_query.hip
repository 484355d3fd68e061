// Query shapes of Table III beyond the single-key windowed group-by:
//  * composite group keys (LR2S groups by highway, direction and segment),
//  * HAVING on an aggregate (LR2S keeps the groups whose average is below a
//    bound),
//  * ORDER BY an aggregate within each window (CM1; Table II "Sorting"),
//  * the windowed self-join of LR1 (the stream joined with the rows of its
//    own range/slide window on equal keys).
//
// Method:
//  * A composite key is packed into one int64 per row by mixed radix over
//    the value domain the caller declares for each key column (the schema's
//    domain, e.g. 0..9 highways): the packing is exact, and its order is the
//    lexicographic order of the tuple.  The windowed group-by then runs on the
//    packed column unchanged, and the finishing pass unpacks the keys.
//  * HAVING is a stable compaction of the groups (tile counts, one scan,
//    ballot-ranked writes).
//  * Sorting is a stable least-significant-digit radix sort of element ids, 8
//    bits per pass: tile histograms, one scan, and a scatter that ranks equal
//    digits within a wave by eight ballots (lanes with the same digit are the
//    intersection of the per-bit ballots), waves and rounds in order, so equal
//    digits keep their order.  A pass whose digit is the same for every element
//    copies instead of scattering.
//  * The self-join sorts the passing rows by (key, pane); the rows of one key
//    in one window are then a contiguous run, found by binary search, and
//    every row emits its pairs with each window it lies in.
#include <algorithm>
#include <cstring>

#include "lms_internal.h"

namespace lms {
namespace {

constexpr int kTPB = 256;
constexpr int kTile = 4096;  // elements per tile of the compaction and sort passes
constexpr int kRounds = kTile / kTPB;
constexpr int kScanTPB = 1024;
constexpr uint64_t kSign = 1ull << 63;

// ---- device scans over tile totals -------------------------------------------

// Exclusive scan of n 64-bit values in place (one workgroup); *total = sum.
__device__ void scan_i64_inplace(int64_t* v, int64_t n, int64_t* total) {
  __shared__ int64_t wsum[kScanTPB / 64 + 1];
  const int64_t per = (n + kScanTPB - 1) / kScanTPB;
  const int64_t lo = (int64_t)threadIdx.x * per;
  const int64_t hi = min(n, lo + per);
  int64_t s = 0;
  for (int64_t i = lo; i < hi; ++i) s += v[i];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int64_t x = s;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int64_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) wsum[wave] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t run = 0;
    for (int w = 0; w < kScanTPB / 64; ++w) {
      const int64_t t = wsum[w];
      wsum[w] = run;
      run += t;
    }
    wsum[kScanTPB / 64] = run;
  }
  __syncthreads();
  int64_t run = wsum[wave] + x - s;
  for (int64_t i = lo; i < hi; ++i) {
    const int64_t t = v[i];
    v[i] = run;
    run += t;
  }
  if (threadIdx.x == 0) *total = wsum[kScanTPB / 64];
  __syncthreads();
}

__device__ __forceinline__ int64_t ntiles_of(int64_t n) { return (n + kTile - 1) / kTile; }

// ---- stable LSD radix sort of element ids ------------------------------------

// One 8-bit pass: digit of element id e = ((field[e] ^ flip) >> shift) & 255.
struct SortPass {
  const uint64_t* field;
  uint64_t flip;
  int32_t shift;
  int32_t reserved;
  const int64_t* d_n;  // element count (device)
  const uint32_t* src;  // ids in the current order
  uint32_t* dst;
  uint32_t* hist;      // [256][tiles]: digit counts, then their exclusive scan
  int32_t* trivial;    // set by the scan when every element has the same digit
};

__device__ __forceinline__ uint32_t digit_of(const SortPass& p, uint32_t id) {
  return (uint32_t)(((p.field[id] ^ p.flip) >> p.shift) & 255u);
}

__global__ __launch_bounds__(kTPB) void k_rs_hist(SortPass p) {
  __shared__ uint32_t h[256];
  const int64_t n = *p.d_n, nt = ntiles_of(n);
  for (int64_t t = blockIdx.x; t < nt; t += gridDim.x) {
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t lo = t * kTile, hi = min(n, lo + kTile);
    for (int64_t e = lo + threadIdx.x; e < hi; e += kTPB) atomicAdd(&h[digit_of(p, p.src[e])], 1u);
    __syncthreads();
    p.hist[(int64_t)threadIdx.x * nt + t] = h[threadIdx.x];
    __syncthreads();
  }
}

__global__ __launch_bounds__(kScanTPB) void k_rs_scan(SortPass p) {
  const int64_t n = *p.d_n, nt = ntiles_of(n);
  __shared__ uint32_t nz;
  if (threadIdx.x == 0) nz = 0;
  __syncthreads();
  // digits holding elements: one alone means the pass keeps the order
  if (threadIdx.x < 256) {
    bool any = false;
    for (int64_t t = 0; t < nt && !any; ++t) any = p.hist[(int64_t)threadIdx.x * nt + t] != 0;
    if (any) atomicAdd(&nz, 1u);
  }
  const int64_t m = 256 * nt;
  const int64_t per = (m + kScanTPB - 1) / kScanTPB;
  const int64_t lo = (int64_t)threadIdx.x * per, hi = min(m, lo + per);
  uint32_t s = 0;
  for (int64_t i = lo; i < hi; ++i) s += p.hist[i];
  __shared__ uint32_t scratch[kScanTPB / 64 + 1];
  uint32_t total;
  uint32_t run = block_excl_scan<kScanTPB>(s, scratch, &total);
  for (int64_t i = lo; i < hi; ++i) {
    const uint32_t c = p.hist[i];
    p.hist[i] = run;
    run += c;
  }
  if (threadIdx.x == 0) *p.trivial = nz <= 1 ? 1 : 0;
}

__global__ __launch_bounds__(kTPB) void k_rs_scatter(SortPass p) {
  __shared__ uint32_t base[256];
  __shared__ uint32_t wcnt[kTPB / 64][256];
  const int64_t n = *p.d_n, nt = ntiles_of(n);
  if (*p.trivial) {  // every element has the same digit: the order stays
    for (int64_t e = (int64_t)blockIdx.x * kTPB + threadIdx.x; e < n; e += (int64_t)gridDim.x * kTPB)
      p.dst[e] = p.src[e];
    return;
  }
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t below = (1ull << lane) - 1;
  for (int64_t t = blockIdx.x; t < nt; t += gridDim.x) {
    base[threadIdx.x] = p.hist[(int64_t)threadIdx.x * nt + t];
    for (int w = 0; w < kTPB / 64; ++w) wcnt[w][threadIdx.x] = 0;
    __syncthreads();
    const int64_t lo = t * kTile;
    for (int r = 0; r < kRounds; ++r) {
      const int64_t e = lo + (int64_t)r * kTPB + threadIdx.x;
      const bool valid = e < n;
      const uint32_t id = valid ? p.src[e] : 0u;
      const uint32_t d = valid ? digit_of(p, id) : 0u;
      // lanes of this wave holding the same digit
      uint64_t same = __ballot(valid);
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t bal = __ballot(valid && bit);
        same &= bit ? bal : ~bal;
      }
      const uint32_t rank = (uint32_t)__popcll(same & below);
      if (valid && rank == 0) wcnt[wave][d] = (uint32_t)__popcll(same);
      __syncthreads();
      if (valid) {
        uint32_t pos = base[d] + rank;
        for (uint32_t w = 0; w < wave; ++w) pos += wcnt[w][d];
        p.dst[pos] = id;
      }
      __syncthreads();
      uint32_t add = 0;
      for (int w = 0; w < kTPB / 64; ++w) {
        add += wcnt[w][threadIdx.x];
        wcnt[w][threadIdx.x] = 0;
      }
      base[threadIdx.x] += add;
      __syncthreads();
    }
  }
}

// Host: sorts ids[0..n) (n on the device, at most cap) stably by the given
// fields, least significant first: each field is (array, xor flip, bits),
// sorted over its low `bits` bits.  ids ends in `a` or `b`; returns which.
struct SortField {
  const uint64_t* field;
  uint64_t flip;
  int bits;
};

struct SortWs {
  uint32_t* a;
  uint32_t* b;
  uint32_t* hist;
  int32_t* trivial;
};

size_t sort_ws_bytes(int64_t cap) {
  WsCarver c(nullptr);
  c.take<uint32_t>((size_t)std::max<int64_t>(1, cap));
  c.take<uint32_t>((size_t)std::max<int64_t>(1, cap));
  c.take<uint32_t>((size_t)256 * std::max<int64_t>(1, (cap + kTile - 1) / kTile));
  c.take<int32_t>(4);
  return c.size();
}

SortWs carve_sort(WsCarver& c, int64_t cap) {
  SortWs s;
  s.a = c.take<uint32_t>((size_t)std::max<int64_t>(1, cap));
  s.b = c.take<uint32_t>((size_t)std::max<int64_t>(1, cap));
  s.hist = c.take<uint32_t>((size_t)256 * std::max<int64_t>(1, (cap + kTile - 1) / kTile));
  s.trivial = c.take<int32_t>(4);
  return s;
}

int num_cus_q() {
  static int n = 0;
  if (n == 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
      n = v;
    else
      n = 256;
  }
  return n;
}

// ids must already hold the elements in `s.a`; returns the buffer holding the result.
uint32_t* radix_sort(const SortWs& s, const int64_t* d_n, int64_t cap, const SortField* fields, int nfields,
                     hipStream_t st) {
  uint32_t* src = s.a;
  uint32_t* dst = s.b;
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((cap + kTile - 1) / kTile, 4 * num_cus_q()));
  for (int f = 0; f < nfields; ++f) {
    for (int shift = 0; shift < fields[f].bits; shift += 8) {
      SortPass p{};
      p.field = fields[f].field;
      p.flip = fields[f].flip;
      p.shift = shift;
      p.d_n = d_n;
      p.src = src;
      p.dst = dst;
      p.hist = s.hist;
      p.trivial = s.trivial;
      LMS_LAUNCH("k_rs_hist", k_rs_hist, dim3(grid), dim3(kTPB), 0, st, p);
      LMS_LAUNCH("k_rs_scan", k_rs_scan, dim3(1), dim3(kScanTPB), 0, st, p);
      LMS_LAUNCH("k_rs_scatter", k_rs_scatter, dim3(grid), dim3(kTPB), 0, st, p);
      std::swap(src, dst);
    }
  }
  return src;
}

// Identity ids 0..n-1.
__global__ void k_iota(uint32_t* ids, const int64_t* d_n) {
  const int64_t n = *d_n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x)
    ids[e] = (uint32_t)e;
}

// ---- composite keys ------------------------------------------------------------

constexpr int kMaxKeys = 4;

struct PackArgs {
  Query q;
  int32_t nkey;
  int32_t kcol[kMaxKeys];
  int64_t klo[kMaxKeys];
  int64_t khi[kMaxKeys];
  uint64_t kmul[kMaxKeys];  // mixed-radix weight of key part j
  int64_t* packed;
  int64_t* d_pack;  // [1]: LMS_ERANGE when a passing row's key lies outside its domain
};

__global__ void k_q_init(int64_t* d_pack) {
  if (threadIdx.x < 2) d_pack[threadIdx.x] = 0;
}

// packed[i] = sum_j (key_j[i] - lo_j) * mul_j for a passing row (0 otherwise).
__global__ __launch_bounds__(kTPB) void k_q_pack(PackArgs a) {
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * kTPB + threadIdx.x; i < a.q.nrows; i += (int64_t)gridDim.x * kTPB) {
    uint64_t v = 0;
    if (row_passes(a.q, i)) {
      for (int j = 0; j < a.nkey; ++j) {
        const int c = a.kcol[j];
        const int64_t x = load_i64(a.q.col[c], a.q.dt[c], i);
        if (x < a.klo[j] || x > a.khi[j]) bad = true;
        else v += (uint64_t)(x - a.klo[j]) * a.kmul[j];
      }
    }
    a.packed[i] = (int64_t)v;
  }
  if (bad) set_device_status(a.d_pack, LMS_ERANGE);
}

// ---- HAVING, key unpacking and ordering ------------------------------------------

struct FinishArgs {
  // groups of the window aggregation (packed key when nkey > 1)
  const int64_t* gkey;
  const int64_t* gws;
  const void* gagg[kMaxAggs];
  const int64_t* d_inner;  // [0] groups, [1] status
  const int64_t* d_pack;   // [1] status of the key packing (0 without composite keys)
  int64_t cap;
  int32_t nagg;
  int32_t afn[kMaxAggs];
  int32_t has_having;
  int32_t hagg, hop;
  int64_t hival;
  double hfval;
  int32_t nkey;
  int32_t packed;  // keys are packed (nkey > 1)
  int64_t klo[kMaxKeys];
  uint64_t kmul[kMaxKeys];
  uint64_t krad[kMaxKeys];
  int64_t* tcnt;  // per-tile kept counts, then offsets; [tiles] = total
  int64_t* d_total;
  // destination: either the caller's columns (keys unpacked) or the staging
  // arrays of an ordered query (packed key, window start, raw aggregates)
  int32_t staged;
  int64_t* okey[kMaxKeys];
  int64_t* ows;
  void* oagg[kMaxAggs];
  int64_t* d_count;  // the caller's count pair
};

__device__ __forceinline__ int64_t finish_groups(const FinishArgs& a) {
  const int64_t g = a.d_inner[0];
  return g < a.cap ? g : a.cap;
}

__device__ __forceinline__ bool keep_group(const FinishArgs& a, int64_t g) {
  if (!a.has_having) return true;
  if (a.afn[a.hagg] == LMS_AVG) return compare<double>(((const double*)a.gagg[a.hagg])[g], a.hop, a.hfval);
  return compare<int64_t>(((const int64_t*)a.gagg[a.hagg])[g], a.hop, a.hival);
}

__global__ __launch_bounds__(kTPB) void k_q_count(FinishArgs a) {
  const int64_t G = finish_groups(a), nt = ntiles_of(G);
  __shared__ uint32_t s;
  for (int64_t t = blockIdx.x; t < nt; t += gridDim.x) {
    if (threadIdx.x == 0) s = 0;
    __syncthreads();
    uint32_t c = 0;
    for (int64_t g = t * kTile + threadIdx.x; g < min(G, (t + 1) * kTile); g += kTPB) c += keep_group(a, g) ? 1u : 0u;
    atomicAdd(&s, c);
    __syncthreads();
    if (threadIdx.x == 0) a.tcnt[t] = s;
    __syncthreads();
  }
}

__global__ __launch_bounds__(kScanTPB) void k_q_scan(FinishArgs a) {
  const int64_t G = finish_groups(a);
  scan_i64_inplace(a.tcnt, ntiles_of(G), a.d_total);
  if (threadIdx.x == 0) {
    a.d_count[0] = *a.d_total;
    const int64_t st = a.d_pack[1] != 0 ? a.d_pack[1] : a.d_inner[1];
    a.d_count[1] = st != 0 ? st : (a.d_inner[0] > a.cap ? LMS_ECAPACITY : 0);
  }
}

__device__ __forceinline__ void unpack_keys(const FinishArgs& a, int64_t key, int64_t (&k)[kMaxKeys]) {
  if (!a.packed) {
    k[0] = key;
    return;
  }
  const uint64_t v = (uint64_t)key;
  for (int j = 0; j < a.nkey; ++j) k[j] = a.klo[j] + (int64_t)((v / a.kmul[j]) % a.krad[j]);
}

// Kept groups in order: the tile's offset plus ballot ranks of the waves in
// turn (each wave walks its stretch of the tile).
__global__ __launch_bounds__(kTPB) void k_q_write(FinishArgs a) {
  const int64_t G = finish_groups(a), nt = ntiles_of(G);
  __shared__ uint32_t wtot[kTPB / 64];
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t below = (1ull << lane) - 1;
  constexpr int kPerWave = kTile / (kTPB / 64);
  for (int64_t t = blockIdx.x; t < nt; t += gridDim.x) {
    const int64_t w0 = t * kTile + (int64_t)wave * kPerWave;
    uint32_t mine = 0;
    for (int64_t b = w0; b < w0 + kPerWave; b += 64) {
      const int64_t g = b + lane;
      mine += (uint32_t)__popcll(__ballot(g < G && keep_group(a, g)));
    }
    if (lane == 0) wtot[wave] = mine;
    __syncthreads();
    int64_t run = a.tcnt[t];
    for (uint32_t w = 0; w < wave; ++w) run += wtot[w];
    for (int64_t b = w0; b < w0 + kPerWave; b += 64) {
      const int64_t g = b + lane;
      const bool keep = g < G && keep_group(a, g);
      const uint64_t m = __ballot(keep);
      const int64_t r = run + __popcll(m & below);
      run += __popcll(m);
      if (!keep) continue;
      if (a.staged) {
        a.okey[0][r] = a.gkey[g];
      } else {
        int64_t k[kMaxKeys];
        unpack_keys(a, a.gkey[g], k);
        for (int j = 0; j < a.nkey; ++j) a.okey[j][r] = k[j];
      }
      a.ows[r] = a.gws[g];
      for (int k = 0; k < a.nagg; ++k) ((int64_t*)a.oagg[k])[r] = ((const int64_t*)a.gagg[k])[g];
    }
    __syncthreads();
  }
}

// Sort fields of an ordered query, in order-preserving unsigned form: the
// aggregate (descending: complemented), and the window start (sign flipped).
struct OrderArgs {
  const int64_t* skey;  // staged packed keys (nonnegative)
  const int64_t* sws;
  const void* sagg;     // staged ordering aggregate
  int32_t is_double, descending;
  const int64_t* d_n;
  uint64_t* fval;
  uint64_t* fws;
};

__global__ void k_q_fields(OrderArgs o) {
  const int64_t n = *o.d_n;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
    uint64_t b = ((const uint64_t*)o.sagg)[e];
    if (o.is_double) b = (b & kSign) ? ~b : (b | kSign);  // IEEE order as unsigned order
    else b ^= kSign;
    o.fval[e] = o.descending ? ~b : b;
    o.fws[e] = (uint64_t)o.sws[e] ^ kSign;
  }
}

// Rows in sorted order into the caller's columns (keys unpacked).
__global__ void k_q_gather(FinishArgs a, const uint32_t* ids, const int64_t* skey, const int64_t* sws) {
  const int64_t n = a.d_count[0];
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t e = ids[r];
    int64_t k[kMaxKeys];
    unpack_keys(a, skey[e], k);
    for (int j = 0; j < a.nkey; ++j) a.okey[j][r] = k[j];
    a.ows[r] = sws[e];
    for (int q = 0; q < a.nagg; ++q) ((int64_t*)a.oagg[q])[r] = ((const int64_t*)a.gagg[q])[e];
  }
}

// ---- windowed self-join -----------------------------------------------------------

struct JoinArgs {
  Query q;
  int32_t key_col, ts_col;
  int64_t len, slide, origin, pane, R, W;
  int64_t* d_m;        // [0] passing rows, [1] base pane (a multiple of R)
  uint32_t* row;       // passing row ids
  uint64_t* fkey;      // key ^ sign bit
  uint64_t* fpane;     // pane relative to the base pane
  // sorted by (key, pane)
  const uint32_t* ids;
  uint32_t* srow;
  uint64_t* skey;
  uint64_t* spane;
  int64_t* cnt;        // pairs per sorted row, then offsets
  int64_t* d_total;
  int64_t* oss;
  uint32_t* ol;
  uint32_t* oa;
  int64_t cap;
  int64_t* d_count;
};

__global__ void k_sj_init(JoinArgs a) {
  if (threadIdx.x != 0) return;
  a.d_m[0] = 0;
  int64_t b0 = 0;
  if (a.q.nrows > 0) {
    const int64_t q0 = floor_div(load_i64(a.q.col[a.ts_col], a.q.dt[a.ts_col], 0) - a.origin, a.pane);
    b0 = a.R * floor_div(q0 - (int64_t(1) << 30), a.R);
  }
  a.d_m[1] = b0;
  a.d_count[0] = 0;
  a.d_count[1] = 0;
}

// Passing rows, in any order (one output reservation per wave).
__global__ __launch_bounds__(kTPB) void k_sj_select(JoinArgs a) {
  const uint32_t lane = threadIdx.x & 63;
  const int64_t b0 = a.d_m[1];
  bool bad = false;
  for (int64_t base = (int64_t)blockIdx.x * kTPB; base < a.q.nrows; base += (int64_t)gridDim.x * kTPB) {
    const int64_t i = base + threadIdx.x;
    const bool ok = i < a.q.nrows && row_passes(a.q, i);
    const uint64_t m = __ballot(ok);
    uint64_t at = 0;
    if (lane == 0 && m) at = (uint64_t)atomicAdd((unsigned long long*)&a.d_m[0], (unsigned long long)__popcll(m));
    at = (uint64_t)__shfl((long long)at, 0, 64);
    if (!ok) continue;
    const uint64_t e = at + __popcll(m & ((1ull << lane) - 1));
    const int64_t rel = floor_div(load_i64(a.q.col[a.ts_col], a.q.dt[a.ts_col], i) - a.origin, a.pane) - b0;
    if (rel < 0 || rel >= (int64_t(1) << 31)) bad = true;
    a.row[e] = (uint32_t)i;
    a.fkey[e] = (uint64_t)load_i64(a.q.col[a.key_col], a.q.dt[a.key_col], i) ^ kSign;
    a.fpane[e] = (uint64_t)(rel < 0 ? 0 : rel);
  }
  if (bad) set_device_status(a.d_count, LMS_ERANGE);
}

__global__ void k_sj_gather(JoinArgs a) {
  const int64_t m = a.d_m[0];
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < m; p += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t e = a.ids[p];
    a.srow[p] = a.row[e];
    a.skey[p] = a.fkey[e];
    a.spane[p] = a.fpane[e];
  }
}

// First position in [lo, hi) whose value is >= x (v nondecreasing there).
__device__ __forceinline__ int64_t lower_bound_u64(const uint64_t* v, int64_t lo, int64_t hi, uint64_t x) {
  while (lo < hi) {
    const int64_t mid = lo + ((hi - lo) >> 1);
    if (v[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// The rows of the key of sorted position p in window w (relative index):
// positions with pane in [w R, w R + W) inside the key's run [rs, re).
__device__ __forceinline__ void window_run(const JoinArgs& a, int64_t rs, int64_t re, int64_t w, int64_t* lo,
                                           int64_t* hi) {
  const int64_t p0 = w * a.R, p1 = p0 + a.W;
  *lo = lower_bound_u64(a.spane, rs, re, (uint64_t)(p0 < 0 ? 0 : p0));
  *hi = lower_bound_u64(a.spane, rs, re, (uint64_t)(p1 < 0 ? 0 : p1));
}

__device__ __forceinline__ void key_run(const JoinArgs& a, int64_t m, int64_t p, int64_t* rs, int64_t* re) {
  const uint64_t k = a.skey[p];
  *rs = lower_bound_u64(a.skey, 0, p, k);
  *re = k == ~0ull ? m : lower_bound_u64(a.skey, p, m, k + 1);
}

__global__ void k_sj_count(JoinArgs a) {
  const int64_t m = a.d_m[0];
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < m; p += (int64_t)gridDim.x * blockDim.x) {
    int64_t rs, re;
    key_run(a, m, p, &rs, &re);
    const int64_t q = (int64_t)a.spane[p];
    const int64_t wf = floor_div(q - a.W, a.R) + 1, wl = floor_div(q, a.R);
    int64_t c = 0;
    for (int64_t w = wf; w <= wl; ++w) {
      int64_t lo, hi;
      window_run(a, rs, re, w, &lo, &hi);
      c += hi - lo;
    }
    a.cnt[p] = c;
  }
}

__global__ __launch_bounds__(kScanTPB) void k_sj_scan(JoinArgs a) {
  scan_i64_inplace(a.cnt, a.d_m[0], a.d_total);
  if (threadIdx.x == 0) a.d_count[0] = *a.d_total;
}

__global__ void k_sj_write(JoinArgs a) {
  const int64_t m = a.d_m[0], b0 = a.d_m[1];
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < m; p += (int64_t)gridDim.x * blockDim.x) {
    int64_t rs, re;
    key_run(a, m, p, &rs, &re);
    const int64_t q = (int64_t)a.spane[p];
    const int64_t wf = floor_div(q - a.W, a.R) + 1, wl = floor_div(q, a.R);
    int64_t o = a.cnt[p];
    for (int64_t w = wf; w <= wl; ++w) {
      int64_t lo, hi;
      window_run(a, rs, re, w, &lo, &hi);
      const int64_t ws = a.origin + (w + b0 / a.R) * a.slide;
      for (int64_t x = lo; x < hi; ++x, ++o) {
        if (o >= a.cap) continue;
        a.oss[o] = ws;
        a.ol[o] = a.srow[p];
        a.oa[o] = a.srow[x];
      }
    }
  }
}

int64_t gcd_q(int64_t x, int64_t y) {
  while (y) {
    const int64_t t = x % y;
    x = y;
    y = t;
  }
  return x;
}

unsigned grid_for(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + kTPB - 1) / kTPB, 8 * num_cus_q()));
}

// Workspace of a windowed query: the packed key column, the groups of the
// window aggregation, tile counts, the ordered query's staging and sort, and
// the aggregation's own workspace.
struct QueryWs {
  int64_t* packed;
  int64_t* gkey;
  int64_t* gws;
  int64_t* gagg[kMaxAggs];
  int64_t* d_inner;
  int64_t* d_pack;
  int64_t* tcnt;
  int64_t* d_total;
  int64_t* skey;
  int64_t* sws;
  int64_t* sagg[kMaxAggs];
  uint64_t* fval;
  uint64_t* fws;
  SortWs sort;
  void* wa;
  size_t wa_bytes;
};

size_t carve_query(void* base, int64_t n, int nkey, int nagg, int64_t cap, bool ordered, size_t wa_bytes,
                   QueryWs* w) {
  WsCarver c(base);
  const size_t capz = (size_t)std::max<int64_t>(1, cap);
  QueryWs q{};
  q.packed = c.take<int64_t>(nkey > 1 ? (size_t)std::max<int64_t>(1, n) : 1);
  q.gkey = c.take<int64_t>(capz);
  q.gws = c.take<int64_t>(capz);
  for (int k = 0; k < nagg; ++k) q.gagg[k] = c.take<int64_t>(capz);
  q.d_inner = c.take<int64_t>(2);
  q.d_pack = c.take<int64_t>(2);
  q.tcnt = c.take<int64_t>((capz + kTile - 1) / kTile + 1);
  q.d_total = c.take<int64_t>(1);
  if (ordered) {
    q.skey = c.take<int64_t>(capz);
    q.sws = c.take<int64_t>(capz);
    for (int k = 0; k < nagg; ++k) q.sagg[k] = c.take<int64_t>(capz);
    q.fval = c.take<uint64_t>(capz);
    q.fws = c.take<uint64_t>(capz);
    q.sort = carve_sort(c, cap);
  }
  q.wa = c.take<char>(wa_bytes);
  q.wa_bytes = wa_bytes;
  if (w) *w = q;
  return c.size();
}

// Validates the key parts; fills mixed-radix weights (the first part most
// significant, so packed order is the tuple's lexicographic order).
int key_weights(const lms_batch* in, const lms_keypart* keys, int32_t nkey, uint64_t* mul, uint64_t* rad) {
  if (!keys || nkey < 1 || nkey > kMaxKeys) return set_error(LMS_EINVAL, "nkey must be in [1, %d]", kMaxKeys);
  unsigned __int128 prod = 1;
  for (int j = nkey - 1; j >= 0; --j) {
    const int c = keys[j].col;
    if (c < 0 || c >= in->ncols) return set_error(LMS_EINVAL, "key part %d column %d out of range", j, c);
    const int dt = in->cols[c].dtype;
    if (dt != LMS_I32 && dt != LMS_I64) return set_error(LMS_EINVAL, "key part %d must be an integer column", j);
    if (nkey == 1) break;
    if (keys[j].hi < keys[j].lo) return set_error(LMS_EINVAL, "key part %d has hi < lo", j);
    const unsigned __int128 r = (unsigned __int128)((__int128)keys[j].hi - (__int128)keys[j].lo + 1);
    mul[j] = (uint64_t)prod;
    rad[j] = (uint64_t)r;
    prod *= r;
    if (prod > ((unsigned __int128)1 << 62))
      return set_error(LMS_EINVAL, "the key domains span more than 2^62 tuples");
  }
  return LMS_OK;
}

}  // namespace
}  // namespace lms

using namespace lms;

extern "C" size_t lms_window_query_workspace(const lms_batch* in, const lms_keypart* keys, int32_t nkey,
                                             const lms_window* w, const lms_agg* aggs, int32_t nagg, int32_t ordered,
                                             int64_t cap) {
  if (!in || !keys || nkey < 1 || nkey > kMaxKeys || nagg < 0 || nagg > kMaxAggs || cap < 0) return 0;
  const int key_col = nkey > 1 ? in->ncols : keys[0].col;
  // the aggregation sees the batch with the packed key appended
  lms_col cols[kMaxCols + 1];
  if (in->ncols > kMaxCols || !in->cols) return 0;
  for (int c = 0; c < in->ncols; ++c) cols[c] = in->cols[c];
  cols[in->ncols] = lms_col{nullptr, LMS_I64, 0};
  const lms_batch in2{cols, in->ncols + (nkey > 1 ? 1 : 0), 0, in->nrows};
  const size_t wa = lms_window_agg_workspace(&in2, key_col, w, aggs, nagg);
  if (wa == 0) return 0;
  return carve_query(nullptr, in->nrows, nkey, nagg, cap, ordered != 0, wa, nullptr);
}

extern "C" int lms_window_query(const lms_batch* in, const lms_pred* preds, int32_t npred, const lms_proj* projs,
                                int32_t nproj, const lms_keypart* keys, int32_t nkey, const lms_window* w,
                                const lms_agg* aggs, int32_t nagg, const lms_having* having, const lms_order* order,
                                const lms_qgroups* out, int64_t* d_count, void* workspace, size_t ws_bytes,
                                lms_stream stream) {
  if (!in || !w || !out || !d_count) return set_error(LMS_EINVAL, "NULL argument");
  if (in->ncols < 0 || in->ncols > kMaxCols || (in->ncols > 0 && !in->cols))
    return set_error(LMS_EINVAL, "bad input batch");
  if (nkey > 1 && in->ncols + 1 > kMaxCols)
    return set_error(LMS_EINVAL, "a composite key needs a free column slot (at most %d input columns)", kMaxCols - 1);
  uint64_t mul[kMaxKeys] = {}, rad[kMaxKeys] = {};
  int rc = key_weights(in, keys, nkey, mul, rad);
  if (rc) return rc;
  if (nagg < 0 || nagg > kMaxAggs || (nagg > 0 && !aggs)) return set_error(LMS_EINVAL, "bad aggregates");
  if (out->cap < 0 || !out->keys || (out->cap > 0 && !out->wstart) || (nagg > 0 && !out->aggs))
    return set_error(LMS_EINVAL, "bad output groups");
  for (int j = 0; j < nkey; ++j)
    if (out->cap > 0 && !out->keys[j]) return set_error(LMS_EINVAL, "output key column %d is NULL", j);
  for (int k = 0; k < nagg; ++k)
    if (out->cap > 0 && !out->aggs[k]) return set_error(LMS_EINVAL, "output aggregate %d is NULL", k);
  if (having && (having->agg < 0 || having->agg >= nagg || having->op < LMS_LT || having->op > LMS_NE))
    return set_error(LMS_EINVAL, "HAVING names aggregate %d of %d or a bad comparison", having ? having->agg : -1,
                     nagg);
  if (order && (order->agg < 0 || order->agg >= nagg)) return set_error(LMS_EINVAL, "ORDER BY names a bad aggregate");
  const bool packed = nkey > 1;
  const int key_col = packed ? in->ncols : keys[0].col;
  // the batch the aggregation sees: the input columns, then the packed key;
  // aggregates over projected columns move one index up
  lms_col cols[kMaxCols + 1];
  for (int c = 0; c < in->ncols; ++c) cols[c] = in->cols[c];
  lms_agg aggs2[kMaxAggs];
  for (int k = 0; k < nagg; ++k) {
    aggs2[k] = aggs[k];
    if (packed && aggs[k].fn != LMS_COUNT && aggs[k].col >= in->ncols) aggs2[k].col += 1;
  }
  const size_t need = lms_window_query_workspace(in, keys, nkey, w, aggs, nagg, order ? 1 : 0, out->cap);
  if (need == 0) return set_error(LMS_EINVAL, "bad windowed query");
  if (!workspace || ws_bytes < need)
    return set_error(LMS_ENOMEM, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
  // the aggregation's workspace size, as lms_window_query_workspace computed it
  cols[in->ncols] = lms_col{nullptr, LMS_I64, 0};
  const lms_batch probe{cols, in->ncols + (packed ? 1 : 0), 0, in->nrows};
  const size_t wa_bytes = lms_window_agg_workspace(&probe, key_col, w, aggs2, nagg);
  QueryWs q;
  carve_query(workspace, in->nrows, nkey, nagg, out->cap, order != nullptr, wa_bytes, &q);
  hipStream_t st = (hipStream_t)stream;
  cols[in->ncols] = lms_col{q.packed, LMS_I64, 0};
  const lms_batch in2{cols, in->ncols + (packed ? 1 : 0), 0, in->nrows};
  void* gaggs[kMaxAggs];
  for (int k = 0; k < nagg; ++k) gaggs[k] = q.gagg[k];
  const lms_groups inner{q.gkey, q.gws, gaggs, out->cap};
  // the aggregation's own validation runs first, so a bad query enqueues nothing
  if (packed) {
    PackArgs pa{};
    rc = build_query(in, preds, npred, projs, nproj, &pa.q);
    if (rc) return rc;
    pa.nkey = nkey;
    for (int j = 0; j < nkey; ++j) {
      pa.kcol[j] = keys[j].col;
      pa.klo[j] = keys[j].lo;
      pa.khi[j] = keys[j].hi;
      pa.kmul[j] = mul[j];
    }
    pa.packed = q.packed;
    pa.d_pack = q.d_pack;  // the aggregation clears its own status word when it starts
    LMS_LAUNCH("k_q_init", k_q_init, dim3(1), dim3(64), 0, st, q.d_pack);
    LMS_LAUNCH("k_q_pack", k_q_pack, dim3(grid_for(in->nrows)), dim3(kTPB), 0, st, pa);
  } else {
    LMS_LAUNCH("k_q_init", k_q_init, dim3(1), dim3(64), 0, st, q.d_pack);
  }
  rc = lms_window_agg(&in2, preds, npred, projs, nproj, key_col, w, aggs2, nagg, &inner, q.d_inner, q.wa, q.wa_bytes,
                      stream);
  if (rc) return rc;
  FinishArgs f{};
  f.gkey = q.gkey;
  f.gws = q.gws;
  for (int k = 0; k < nagg; ++k) {
    f.gagg[k] = q.gagg[k];
    f.afn[k] = aggs[k].fn;
  }
  f.d_inner = q.d_inner;
  f.d_pack = q.d_pack;
  f.cap = out->cap;
  f.nagg = nagg;
  f.has_having = having ? 1 : 0;
  if (having) {
    f.hagg = having->agg;
    f.hop = having->op;
    f.hival = having->ival;
    f.hfval = having->fval;
  }
  f.nkey = nkey;
  f.packed = packed ? 1 : 0;
  for (int j = 0; j < nkey; ++j) {
    f.klo[j] = keys[j].lo;
    f.kmul[j] = mul[j];
    f.krad[j] = rad[j];
  }
  f.tcnt = q.tcnt;
  f.d_total = q.d_total;
  f.d_count = d_count;
  f.staged = order ? 1 : 0;
  if (order) {
    f.okey[0] = q.skey;
    f.ows = q.sws;
    for (int k = 0; k < nagg; ++k) f.oagg[k] = q.sagg[k];
  } else {
    for (int j = 0; j < nkey; ++j) f.okey[j] = out->keys[j];
    f.ows = out->wstart;
    for (int k = 0; k < nagg; ++k) f.oagg[k] = out->aggs[k];
  }
  const unsigned tgrid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((out->cap + kTile - 1) / kTile, 4 * num_cus_q()));
  LMS_LAUNCH("k_q_count", k_q_count, dim3(tgrid), dim3(kTPB), 0, st, f);
  LMS_LAUNCH("k_q_scan", k_q_scan, dim3(1), dim3(kScanTPB), 0, st, f);
  LMS_LAUNCH("k_q_write", k_q_write, dim3(tgrid), dim3(kTPB), 0, st, f);
  if (order) {
    OrderArgs o{};
    o.skey = q.skey;
    o.sws = q.sws;
    o.sagg = q.sagg[order->agg];
    o.is_double = aggs[order->agg].fn == LMS_AVG ? 1 : 0;
    o.descending = order->descending ? 1 : 0;
    o.d_n = d_count;
    o.fval = q.fval;
    o.fws = q.fws;
    LMS_LAUNCH("k_q_fields", k_q_fields, dim3(grid_for(out->cap)), dim3(kTPB), 0, st, o);
    LMS_LAUNCH("k_iota", k_iota, dim3(grid_for(out->cap)), dim3(kTPB), 0, st, q.sort.a, (const int64_t*)d_count);
    // least significant first: the key tuple, the aggregate, the window
    int kbits = 0;
    if (packed) {
      unsigned __int128 prod = 1;
      for (int j = 0; j < nkey; ++j) prod *= rad[j];
      while (kbits < 64 && ((unsigned __int128)1 << kbits) < prod) ++kbits;
    } else {
      kbits = 64;
    }
    const SortField fields[3] = {{(const uint64_t*)q.skey, packed ? 0ull : kSign, (kbits + 7) / 8 * 8},
                                 {q.fval, 0ull, 64},
                                 {q.fws, 0ull, 64}};
    const uint32_t* ids = radix_sort(q.sort, d_count, out->cap, fields, 3, st);
    FinishArgs g = f;
    for (int j = 0; j < nkey; ++j) g.okey[j] = out->keys[j];
    g.ows = out->wstart;
    for (int k = 0; k < nagg; ++k) {
      g.oagg[k] = out->aggs[k];
      g.gagg[k] = q.sagg[k];
    }
    LMS_LAUNCH("k_q_gather", k_q_gather, dim3(grid_for(out->cap)), dim3(kTPB), 0, st, g, ids,
               (const int64_t*)q.skey, (const int64_t*)q.sws);
  }
  return check_hip(hipGetLastError(), "window_query launch");
}

extern "C" size_t lms_window_self_join_workspace(int64_t nrows) {
  if (nrows < 0) return 0;
  const size_t n = (size_t)std::max<int64_t>(1, nrows);
  WsCarver c(nullptr);
  c.take<int64_t>(2);
  c.take<uint32_t>(n);
  c.take<uint64_t>(n);
  c.take<uint64_t>(n);
  c.take<uint32_t>(n);
  c.take<uint64_t>(n);
  c.take<uint64_t>(n);
  c.take<int64_t>(n);
  c.take<int64_t>(1);
  return c.size() + sort_ws_bytes(nrows);
}

extern "C" int lms_window_self_join(const lms_batch* in, const lms_pred* preds, int32_t npred, int32_t key_col,
                                    const lms_window* w, int64_t* out_wstart, uint32_t* out_l, uint32_t* out_a,
                                    int64_t cap, int64_t* d_count, void* workspace, size_t ws_bytes,
                                    lms_stream stream) {
  if (!in || !w || !d_count) return set_error(LMS_EINVAL, "NULL argument");
  if (cap < 0 || (cap > 0 && (!out_wstart || !out_l || !out_a))) return set_error(LMS_EINVAL, "bad output");
  JoinArgs a{};
  int rc = build_query(in, preds, npred, nullptr, 0, &a.q);
  if (rc) return rc;
  if (in->nrows >= (int64_t(1) << 31)) return set_error(LMS_EINVAL, "micro-batch must have < 2^31 rows");
  if (key_col < 0 || key_col >= in->ncols || !(in->cols[key_col].dtype == LMS_I32 || in->cols[key_col].dtype == LMS_I64))
    return set_error(LMS_EINVAL, "key column must be an integer column of the batch");
  if (w->ts_col < 0 || w->ts_col >= in->ncols ||
      !(in->cols[w->ts_col].dtype == LMS_I32 || in->cols[w->ts_col].dtype == LMS_I64))
    return set_error(LMS_EINVAL, "ts column must be an integer column of the batch");
  if (w->len <= 0 || w->len >= (int64_t(1) << 31) || w->slide < 0 || w->slide > w->len)
    return set_error(LMS_EINVAL, "bad window");
  const size_t need = lms_window_self_join_workspace(in->nrows);
  if (!workspace || ws_bytes < need)
    return set_error(LMS_ENOMEM, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
  const int64_t n = in->nrows;
  WsCarver c(workspace);
  a.d_m = c.take<int64_t>(2);
  a.row = c.take<uint32_t>((size_t)std::max<int64_t>(1, n));
  a.fkey = c.take<uint64_t>((size_t)std::max<int64_t>(1, n));
  a.fpane = c.take<uint64_t>((size_t)std::max<int64_t>(1, n));
  a.srow = c.take<uint32_t>((size_t)std::max<int64_t>(1, n));
  a.skey = c.take<uint64_t>((size_t)std::max<int64_t>(1, n));
  a.spane = c.take<uint64_t>((size_t)std::max<int64_t>(1, n));
  a.cnt = c.take<int64_t>((size_t)std::max<int64_t>(1, n));
  a.d_total = c.take<int64_t>(1);
  const SortWs sw = carve_sort(c, n);
  a.key_col = key_col;
  a.ts_col = w->ts_col;
  a.len = w->len;
  a.slide = w->slide == 0 ? w->len : w->slide;
  a.origin = w->origin;
  a.pane = gcd_q(a.len, a.slide);
  a.R = a.slide / a.pane;
  a.W = a.len / a.pane;
  a.oss = out_wstart;
  a.ol = out_l;
  a.oa = out_a;
  a.cap = cap;
  a.d_count = d_count;
  hipStream_t st = (hipStream_t)stream;
  LMS_LAUNCH("k_sj_init", k_sj_init, dim3(1), dim3(64), 0, st, a);
  LMS_LAUNCH("k_sj_select", k_sj_select, dim3(grid_for(n)), dim3(kTPB), 0, st, a);
  LMS_LAUNCH("k_iota", k_iota, dim3(grid_for(n)), dim3(kTPB), 0, st, sw.a, (const int64_t*)a.d_m);
  // least significant first: the pane, then the key
  const SortField fields[2] = {{a.fpane, 0ull, 32}, {a.fkey, 0ull, 64}};
  a.ids = radix_sort(sw, a.d_m, n, fields, 2, st);
  LMS_LAUNCH("k_sj_gather", k_sj_gather, dim3(grid_for(n)), dim3(kTPB), 0, st, a);
  LMS_LAUNCH("k_sj_count", k_sj_count, dim3(grid_for(n)), dim3(kTPB), 0, st, a);
  LMS_LAUNCH("k_sj_scan", k_sj_scan, dim3(1), dim3(kScanTPB), 0, st, a);
  LMS_LAUNCH("k_sj_write", k_sj_write, dim3(grid_for(n)), dim3(kTPB), 0, st, a);
  return check_hip(hipGetLastError(), "window_self_join launch");
}
