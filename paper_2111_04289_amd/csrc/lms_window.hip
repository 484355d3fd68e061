// Windowed hash group-by over tumbling and sliding event-time windows.
//
// Semantics: Table II "Aggregation (Hash)" (with "Expand" for sliding
// windows) under the window model of Table I (SlideTime; 0 = tumbling) and the
// range/slide clauses of Table III.  A row belongs to every window
// [origin + k*slide, origin + k*slide + len) that contains its event time.
//
// Method (MI355X-first; the paper delegates these operators to Spark-Rapids):
//  * Pane indices are stored relative to a base 2^30 panes before the first
//    row's pane, so they and the window indices fit 32 bits.
//  * Pane decomposition replaces Expand: with pane = gcd(len, slide) every
//    window is the union of len/pane consecutive panes, and each row falls in
//    exactly one pane, so the row scan does one insertion per row instead of
//    len/slide.
//  * Device-scope global atomics on gfx950 run at the memory side (tens of
//    G ops/s for the whole chip), so no per-row global atomic is used.  Rows are
//    radix-partitioned by a hash of the key (hist -> scan -> scatter) so that
//    all panes of a key land in one partition, and each partition is
//    aggregated in a workgroup's LDS hash tables, where the sliding windows are
//    also composed from the key's panes and emitted.
//  * Zipf-hot partitions are cut into row pieces aggregated by separate
//    workgroups whose LDS partial tables are flushed as partial records and
//    merged by a second launch.
//  * A partition whose groups exceed the LDS tables is re-aggregated in
//    sub-ranges of a second key hash (halving until it fits).
#include <algorithm>
#include <cstring>
#include <mutex>
#include <type_traits>

#include "lms_internal.h"

namespace lms {
namespace {

constexpr int kScanTPB = 256;
constexpr int kScatterTPB = 256;  // measured: 512 threads per chunk ran slower
constexpr int kAggTPB = 1024;
// Waves per SIMD the aggregation kernels are compiled for: one 1024-thread
// workgroup per CU (what the default 2048-slot LDS tables allow) is 4 waves
// per SIMD, so more independent LDS chains are in flight while each waits.
constexpr int agg_waves(int) { return 4; }
constexpr uint64_t kEmptyKey = 0x8000000000000000ull;
constexpr uint64_t kEmptyGid = ~0ull;
constexpr int kLdsLimit = 160 * 1024;
constexpr int kStackCap = 80;
constexpr int kUnroll = 4;
constexpr int kHistUnroll = 8;
constexpr int64_t kMaxChunk = 65536;  // rows of a scan chunk at most (its pass mask is staged in LDS)
constexpr int kXcds = 8;  // XCDs of an MI355X

struct Item {
  uint32_t p, lo, hi, first;
  uint32_t kp, reserved[3];
};

struct PartInfo {
  uint32_t first, kp, start, reserved;
};

struct WinArgs {
  Query q;
  int32_t key_col, ts_col;
  int32_t quads;  // the predicate and key columns start on 16-byte boundaries
  int32_t emit_only;  // re-emission from an intact workspace: split pieces keep their partial records
  int64_t len, slide, origin, pane, R, W;
  double inv_pane;
  double inv_R;
  int32_t nagg;
  int32_t afn[kMaxAggs];
  int32_t aacc[kMaxAggs];  // accumulator slot of aggregate a (-1 for COUNT)
  int32_t nval;
  int32_t vcol[kMaxAggs];  // extended column staged as value column v
  int32_t vdt[kMaxAggs];   // dtype of staged value column v
  int32_t nacc;
  int32_t accfn[kMaxAggs];   // aggregate function of accumulator slot s
  int32_t accval[kMaxAggs];  // staged value column feeding slot s
  int32_t pbits, nparts, g1, max_items, ek, eg;
  int64_t chunk, rs;
  // workspace
  // [0] base pane B0, [1] items, [2]/[3] work counters, [4] split partitions,
  // [5] device status of the call, [6] kSavedMagic once `saved` holds the
  // call's arguments, [7] 1 while a re-emission's arguments are valid
  int64_t* hdr;
  struct WinArgs* saved;  // [0] the call's own arguments, [1] those of a re-emission
  uint32_t* splits;  // nparts: the partitions split into pieces, in claim order
  uint32_t* H;
  uint32_t* Off;
  uint32_t* Rp;
  PartInfo* pinfo;
  Item* items;
  uint32_t* pfill;  // nparts: partial records reserved so far in each split partition
  uint64_t* pmask;  // (nrows + 63) / 64: which rows pass the predicates (bit r % 64 of word r / 64)
  // staged rows, one record of `rec` bytes per passing row: key (8 B) at 0,
  // 8-byte values, pane (4 B) at pane_off, 4-byte values, padding to 8 B --
  // one contiguous record keeps a partition's short per-chunk segment to one
  // or two cache lines instead of a partial line in each of several arrays
  char* srec;
  int32_t rec, pane_off;
  int32_t voff[kMaxAggs];  // byte offset of staged value column v in a record
  int64_t* pkey;
  uint32_t* ppane;
  uint32_t* pcnt;
  uint64_t* pacc[kMaxAggs];
  // outputs
  int64_t* okey;
  int64_t* ows;
  void* oagg[kMaxAggs];
  int64_t cap;
  int64_t* d_count;
};

// LDS the multi-batch aggregation kernels keep for their copy of the batch
// arguments (static LDS, ahead of the 16-byte-aligned dynamic part)
constexpr int kArgsLds = (int)((sizeof(WinArgs) + 255) / 256 * 256);

__device__ __forceinline__ int part_of(uint64_t h, int pbits) { return pbits ? (int)(h >> (64 - pbits)) : 0; }
__device__ __forceinline__ uint32_t subhash(uint64_t h) { return (uint32_t)(h >> 16); }

// Quotient of rel >= 0 by pane, exact: double estimate then integer fix-up.
__device__ __forceinline__ uint64_t div_pane(uint64_t rel, int64_t pane, double inv) {
  if (rel < (1ull << 52)) {
    uint64_t q = (uint64_t)((double)rel * inv);
    int64_t r = (int64_t)(rel - q * (uint64_t)pane);
    while (r < 0) {
      --q;
      r += pane;
    }
    while (r >= pane) {
      ++q;
      r -= pane;
    }
    return q;
  }
  return rel / (uint64_t)pane;
}

// ---- kernels 1-4: partition rows by key hash --------------------------------

__device__ __forceinline__ void init_batch(const WinArgs& a) {
  {
    a.d_count[0] = 0;
    a.d_count[1] = 0;
    a.hdr[1] = 0;
    a.hdr[2] = 0;  // next aggregation item to claim
    a.hdr[3] = 0;  // next split partition to claim for merging
    a.hdr[4] = 0;  // split partitions
    a.hdr[5] = 0;  // status
    int64_t b0 = 0;
    if (a.q.nrows > 0) {
      const int64_t ts0 = load_i64(a.q.col[a.ts_col], a.q.dt[a.ts_col], 0);
      const int64_t q0 = floor_div(ts0 - a.origin, a.pane);
      b0 = a.R * floor_div(q0 - (int64_t(1) << 30), a.R);
    }
    a.hdr[0] = b0;
  }
}

// Marks a workspace whose `saved` slot holds the arguments of the call that
// filled it (lms_window_agg_emit re-emits from such a workspace).
constexpr int64_t kSavedMagic = 0x4c4d5357494e4147ll;
// Byte offset of the `saved` slot: the header takes the first 256 bytes.
constexpr size_t kSavedOff = 256;

// Device status of a call: the caller's d_count[1], and the workspace header
// for a later re-emission.
__device__ __forceinline__ void win_status(const WinArgs& a, int code) {
  set_device_status(a.d_count, code);
  atomicMin((long long*)&a.hdr[5], (long long)code);
}

// Every thread of the block copies its share of the words (a single thread
// copying the whole struct went through private memory, one word at a time);
// thread 0 then marks the slot valid after the block's barrier.
__device__ __forceinline__ void save_args(const WinArgs& a) {
  const uint32_t* src = (const uint32_t*)&a;
  uint32_t* dst = (uint32_t*)a.saved;
  for (uint32_t i = threadIdx.x; i < sizeof(WinArgs) / 4; i += blockDim.x) dst[i] = src[i];
  __syncthreads();
  if (threadIdx.x == 0) a.hdr[6] = kSavedMagic;
}

__global__ void k_wa_init(WinArgs a) {
  if (threadIdx.x == 0) init_batch(a);
  save_args(a);
}

// Chunk processed by workgroup slot g of a launch over n chunks (slots padded
// to a multiple of 8; a result >= n is a padding slot).  Workgroups are
// dispatched round-robin over the 8 XCDs, so slot g runs on XCD g % 8; giving
// each XCD a contiguous range of chunks puts neighbouring chunks -- which
// share the cache lines of the per-(partition, chunk) count and offset arrays
// and of each partition's staged segments -- in one XCD's L2 at about the same
// time, so their partial-line writes merge there.
__device__ __forceinline__ uint32_t xcd_chunk(uint32_t g, uint32_t n) {
  const uint32_t c8 = (n + kXcds - 1) / kXcds;
  return (g % kXcds) * c8 + g / kXcds;
}

constexpr int kHistQuads = 4;  // quads per thread per step of the histogram

// Pass bits of the rows [g, g + 256) of a wave's quads (lane l holds rows
// g + 4l .. g + 4l + 3 in the low four bits of m; g relative to the chunk):
// each group of 16 lanes ORs its nibbles into one 64-bit word of the chunk's
// LDS mask, written by its first lane.
__device__ __forceinline__ void put_quad_mask(uint64_t* lmask, int64_t g, uint32_t m) {
  const int lane = threadIdx.x & 63;
  uint64_t v = (uint64_t)(m & 0xFu) << (4 * (lane & 15));
#pragma unroll
  for (int d = 1; d < 16; d <<= 1) v |= (uint64_t)__shfl_xor((long long)v, d, 64);
  if ((lane & 15) == 0) lmask[(g >> 6) + (lane >> 4)] = v;
}

// LDS bytes of the histogram kernels: the partition counts, then the pass
// mask of one chunk (written to the workspace once per chunk, so the row
// loop's waits are not held up by stores).
__host__ __device__ inline size_t hist_lds(int nparts, int64_t chunk) {
  return (size_t)((nparts + 1) & ~1) * 4 + (size_t)(chunk + 63) / 64 * 8;
}

template <bool kWide>
__device__ __forceinline__ void hist_quads(const WinArgs& a, const void* kc, const int64_t (&kr)[kHistQuads],
                                           const uint32_t (&m)[kHistQuads], uint32_t* hist) {
  uint64_t k[kHistQuads][4];
  load_quads<kWide, kHistQuads>(kc, kr, k);
#pragma unroll
  for (int u = 0; u < kHistQuads; ++u)
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if ((m[u] >> e) & 1u) {
        const int64_t key = kWide ? (int64_t)k[u][e] : (int64_t)(int32_t)(uint32_t)k[u][e];
        atomicAdd(&hist[part_of(fmix64((uint64_t)key), a.pbits)], 1u);
      }
}

// LDS histogram of the passing rows of chunk w over the partitions.
__device__ void hist_chunk(const WinArgs& a, uint32_t w, uint32_t* hist) {
  uint64_t* const lmask = (uint64_t*)(hist + ((a.nparts + 1) & ~1));  // the chunk's pass words
  for (int p = threadIdx.x; p < a.nparts; p += kScanTPB) hist[p] = 0;
  __syncthreads();
  const int64_t lo = (int64_t)w * a.chunk;
  const int64_t hi = min(a.q.nrows, lo + a.chunk);
  const void* kc = a.q.col[a.key_col];
  const int kdt = a.q.dt[a.key_col];
  int64_t b0 = lo;
  if (a.quads) {
    // row quads (see lms_internal.h): thread t takes rows 4t .. 4t + 3 of
    // each 1024-row block, kHistQuads blocks per step; a quad with no passing
    // row reads the chunk's first quad of keys instead of its own
    for (; b0 + 1024 * kHistQuads <= hi; b0 += 1024 * kHistQuads) {
      int64_t r0[kHistQuads], kr[kHistQuads];
      uint32_t m[kHistQuads];
#pragma unroll
      for (int u = 0; u < kHistQuads; ++u) r0[u] = b0 + u * 1024 + 4 * threadIdx.x;
      quads_pass<kHistQuads>(a.q, r0, m);
#pragma unroll
      for (int u = 0; u < kHistQuads; ++u) put_quad_mask(lmask, b0 - lo + u * 1024 + (threadIdx.x & ~63u) * 4, m[u]);
#pragma unroll
      for (int u = 0; u < kHistQuads; ++u) kr[u] = m[u] ? r0[u] : lo;
      if (wide_dtype(kdt)) hist_quads<true>(a, kc, kr, m, hist);
      else hist_quads<false>(a, kc, kr, m, hist);
    }
  }
  // kHistUnroll rows per thread per step, a wave taking 64 kHistUnroll
  // consecutive rows (64 per load, from a multiple of 64); keys are loaded only
  // for passing rows, so a selective predicate leaves most key lines unread
  const int lane = threadIdx.x & 63;
  for (int64_t b = b0 + (threadIdx.x >> 6) * (64 * kHistUnroll) + lane; b < hi;
       b += (int64_t)kScanTPB * kHistUnroll) {
    bool ok[kHistUnroll];
    int64_t key[kHistUnroll];
    int64_t idx[kHistUnroll];
#pragma unroll
    for (int u = 0; u < kHistUnroll; ++u) {
      idx[u] = b + (int64_t)u * 64;
      ok[u] = idx[u] < hi;
    }
    rows_pass<kHistUnroll>(a.q, idx, ok, lo);
    // the wave's kHistUnroll pass words are consecutive: lane u holds word u
    uint64_t mw = 0;
#pragma unroll
    for (int u = 0; u < kHistUnroll; ++u) {
      const uint64_t bits = __ballot(ok[u]);
      if (lane == u) mw = bits;
    }
    const int64_t wrow = b - lane + (int64_t)lane * 64;  // first row of word `lane`
    if (lane < kHistUnroll && wrow < hi) lmask[(wrow - lo) >> 6] = mw;
    load_i64_rows<kHistUnroll>(kc, kdt, idx, ok, lo, key);
#pragma unroll
    for (int u = 0; u < kHistUnroll; ++u)
      if (ok[u]) atomicAdd(&hist[part_of(fmix64((uint64_t)key[u]), a.pbits)], 1u);
  }
  __syncthreads();
  for (int p = threadIdx.x; p < a.nparts; p += kScanTPB) a.H[(size_t)p * a.g1 + w] = hist[p];
  const int nw = (int)((hi - lo + 63) >> 6);
  for (int i = threadIdx.x; i < nw; i += kScanTPB) gptr(a.pmask)[(lo >> 6) + i] = lmask[i];
  __syncthreads();
}

__global__ __launch_bounds__(kScanTPB) void k_wa_hist(WinArgs a) {
  extern __shared__ uint32_t hist[];
  // the batch header is set here (nothing in this kernel reads it), which
  // saves a launch before the histogram
  if (blockIdx.x == 0 && threadIdx.x == 0) init_batch(a);
  const uint32_t w = xcd_chunk(blockIdx.x, (uint32_t)a.g1);
  if (w >= (uint32_t)a.g1) return;
  hist_chunk(a, w, hist);
}

// Rows per partition.
__device__ void scan1_part(const WinArgs& a, int p, uint32_t* scratch) {
  uint32_t s = 0;
  for (int w = threadIdx.x; w < a.g1; w += kScanTPB) s += a.H[(size_t)p * a.g1 + w];
  s = block_sum<kScanTPB>(s, scratch);
  if (threadIdx.x == 0) a.Rp[p] = s;
}

__global__ __launch_bounds__(kScanTPB) void k_wa_scan1(WinArgs a) {
  __shared__ uint32_t scratch[kScanTPB / 64 + 1];
  scan1_part(a, blockIdx.x, scratch);
}

constexpr int kMaxParts = 4096;  // partitions of one batch (make_plan's bound)
constexpr int64_t kMinParts = 32;  // partitions a batch of 64K rows or more is spread over at least
constexpr int kPlanTPB = 1024;   // threads of the planning workgroup: a few partitions each

// Partition starts and the aggregation work items of one batch (one
// workgroup; r, st, kc, base are kMaxParts-word LDS arrays):
//  * a partition of more than rs rows gives ceil(R / rs) pieces, whose partial
//    records k_wa_merge combines;
//  * a partition of (eg/4, rs] rows is one item;
//  * non-empty partitions of at most eg/4 rows are packed: consecutive ones
//    whose starts fall in the same eg/4-row bucket form one item of at most
//    eg/2 rows -- few enough groups for the LDS table even when every row is a
//    group of its own -- and a larger partition between two of them always
//    starts a new bucket.  Low selectivity or small batches then give few,
//    fuller items instead of thousands of nearly empty ones.
__device__ void plan_items(const WinArgs& a, uint32_t* r, uint32_t* st, uint32_t* kc, uint32_t* base,
                           uint32_t* scratch) {
  const int np = a.nparts;
  const uint32_t rs = (uint32_t)a.rs, pack = (uint32_t)a.eg / 4;
  for (int p = threadIdx.x; p < np; p += kPlanTPB) {
    const uint32_t v = a.Rp[p];
    r[p] = v;
    st[p] = v;
  }
  __syncthreads();
  const uint32_t total = block_scan_array<kPlanTPB>(st, np, scratch);
  for (int p = threadIdx.x; p < np; p += kPlanTPB) {
    const uint32_t v = r[p];
    uint32_t k = 0;
    if (v > rs) {
      k = (v + rs - 1) / rs;
    } else if (v > pack) {
      k = 1;
    } else if (v > 0) {  // packed: the first of its bucket leads the item
      const uint32_t b = st[p] / pack;
      bool leader = true;
      for (int q = p - 1; q >= 0; --q) {
        const uint32_t w = r[q];
        if (w == 0) continue;
        leader = w > pack || st[q] / pack != b;
        break;
      }
      k = leader ? 1 : 0;
    }
    kc[p] = k;
    base[p] = k;
  }
  __syncthreads();
  const uint32_t nitems = block_scan_array<kPlanTPB>(base, np, scratch);
  // Items are claimed in array order, so they are placed longest first (by
  // an estimate of their time): the last claims are then short ones, and the
  // workgroups finish close together.  The estimate (microseconds; measured
  // on the 16M-row sliding query: an unsplit item about 30 + 5 per 1000 rows,
  // a piece about 7 + 3.4) picks one of 64 classes; the order within a class
  // is arbitrary, as is the claim order itself.  The full pieces of a split
  // partition share a class, so they take consecutive slots with one claim.
  // (Plain code over LDS arrays: item records built in lambdas went through
  // private memory.)
  __shared__ uint32_t ccls[64];
  auto cls = [](uint32_t est) { return 63u - min(63u, est); };
  uint32_t* const ihi = base;  // the item start array is not needed any more: end of an unsplit item
  for (int p = threadIdx.x; p < np; p += kPlanTPB) {
    const uint32_t v = r[p], s0 = st[p];
    uint32_t hi = s0 + v;
    if (v > 0 && v <= pack && kc[p] != 0) {  // a packed item extends over the rest of its bucket
      const uint32_t b = s0 / pack;
      int q = p + 1;
      while (q < np && (r[q] == 0 || (r[q] <= pack && st[q] / pack == b))) ++q;
      hi = q < np ? st[q] : total;
    }
    ihi[p] = hi;
  }
  if (threadIdx.x < 64) ccls[threadIdx.x] = 0;
  __syncthreads();
  for (int p = threadIdx.x; p < np; p += kPlanTPB) {
    const uint32_t v = r[p], k = kc[p];
    if (k == 0) continue;
    if (v > rs) {
      if (k > 1) atomicAdd(&ccls[cls(7u + rs / 300u)], k - 1);
      atomicAdd(&ccls[cls(7u + (v - (k - 1) * rs) / 300u)], 1u);
    } else {
      atomicAdd(&ccls[cls(30u + (ihi[p] - st[p]) / 200u)], 1u);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int c = 0; c < 64; ++c) {
      const uint32_t t = ccls[c];
      ccls[c] = run;
      run += t;
    }
  }
  __syncthreads();
  auto put = [&](uint32_t at, uint32_t p, uint32_t lo, uint32_t hi, uint32_t kp) {
    uint4* const d = (uint4*)&a.items[at];
    d[0] = make_uint4(p, lo, hi, 0u);
    d[1] = make_uint4(kp, 0u, 0u, 0u);
  };
  for (int p = threadIdx.x; p < np; p += kPlanTPB) {
    const uint32_t v = r[p], k = kc[p], s0 = st[p];
    if (k > 0) {
      if (v > rs) {
        if (k > 1) {
          const uint32_t at = atomicAdd(&ccls[cls(7u + rs / 300u)], k - 1);
          for (uint32_t j = 0; j + 1 < k; ++j) put(at + j, (uint32_t)p, s0 + j * rs, s0 + (j + 1) * rs, k);
        }
        put(atomicAdd(&ccls[cls(7u + (v - (k - 1) * rs) / 300u)], 1u), (uint32_t)p, s0 + (k - 1) * rs, s0 + v, k);
      } else {
        put(atomicAdd(&ccls[cls(30u + (ihi[p] - s0) / 200u)], 1u), (uint32_t)p, s0, ihi[p], 1u);
      }
    }
    a.pinfo[p].first = 0;
    a.pinfo[p].kp = k;
    a.pinfo[p].start = s0;
    a.pinfo[p].reserved = 0;
    a.pfill[p] = 0;
  }
  __syncthreads();
  // list of the split partitions (the merge pass claims them one by one)
  for (int p = threadIdx.x; p < np; p += kPlanTPB) kc[p] = r[p] > rs ? 1u : 0u;
  __syncthreads();
  const uint32_t nsplit = block_scan_array<kPlanTPB>(kc, np, scratch);
  for (int p = threadIdx.x; p < np; p += kPlanTPB)
    if (r[p] > rs) a.splits[kc[p]] = (uint32_t)p;
  if (threadIdx.x == 0) {
    a.hdr[1] = nitems;
    a.hdr[4] = nsplit;
  }
  __syncthreads();
}

__global__ __launch_bounds__(kPlanTPB) void k_wa_scanp(WinArgs a) {
  __shared__ uint32_t r[kMaxParts], st[kMaxParts], kc[kMaxParts], base[kMaxParts];
  __shared__ uint32_t scratch[kPlanTPB / 64 + 1];
  plan_items(a, r, st, kc, base, scratch);
  save_args(a);
}

// Per-(partition, chunk) write offsets: partition start plus an exclusive scan
// of H[p][*] in chunk order (neighbouring chunks run on one XCD, so their
// segments of a partition are adjacent in that XCD's L2).
__device__ void scan2_part(const WinArgs& a, int p, uint32_t* scratch) {
  const uint32_t start = a.pinfo[p].start;
  const int per = (a.g1 + kScanTPB - 1) / kScanTPB;
  const int w0 = threadIdx.x * per;
  const int w1 = min(a.g1, w0 + per);
  const uint32_t* h = a.H + (size_t)p * a.g1;
  uint32_t loc = 0;
  for (int w = w0; w < w1; ++w) loc += h[w];
  uint32_t total;
  uint32_t run = start + block_excl_scan<kScanTPB>(loc, scratch, &total);
  for (int w = w0; w < w1; ++w) {
    const uint32_t c = h[w];
    a.Off[(size_t)p * a.g1 + w] = run;
    run += c;
  }
  __syncthreads();
}

__global__ __launch_bounds__(kScanTPB) void k_wa_scan2(WinArgs a) {
  __shared__ uint32_t scratch[kScanTPB / 64 + 1];
  scan2_part(a, blockIdx.x, scratch);
}

// The three steps above in one workgroup, for a batch of at most kSmallChunks
// chunks (a micro-batch, whose three launches would cost more than their
// work): each wave takes one partition at a time, one chunk per lane, and sums
// (rows per partition) or scans (write offsets) the partition's chunk counts
// with shuffles; the plan sits between the two, as in the separate launches.
constexpr int kSmallChunks = 64;

__global__ __launch_bounds__(kPlanTPB) void k_wa_scans(WinArgs a) {
  __shared__ uint32_t r[kMaxParts], st[kMaxParts], kc[kMaxParts], base[kMaxParts];
  __shared__ uint32_t scratch[kPlanTPB / 64 + 1];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int p = wave; p < a.nparts; p += kPlanTPB / 64) {
    uint32_t s = lane < a.g1 ? a.H[(size_t)p * a.g1 + lane] : 0u;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) s += (uint32_t)__shfl_xor((int)s, d, 64);
    if (lane == 0) a.Rp[p] = s;
  }
  __syncthreads();
  plan_items(a, r, st, kc, base, scratch);  // ends with a barrier: every partition start is set
  for (int p = wave; p < a.nparts; p += kPlanTPB / 64) {
    const uint32_t h = lane < a.g1 ? a.H[(size_t)p * a.g1 + lane] : 0u;
    uint32_t x = h;  // inclusive scan over the lanes
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y = (uint32_t)__shfl_up((int)x, d, 64);
      if (lane >= d) x += y;
    }
    if (lane < a.g1) a.Off[(size_t)p * a.g1 + lane] = a.pinfo[p].start + x - h;
  }
  save_args(a);
}

// Raw bits of staged value column v (int64, or the float's own bits) for rows
// idx[u] where ld[u], U at a time (see load_i64_rows).
template <int U>
__device__ __forceinline__ void staged_rows(const WinArgs& a, int v, const int64_t (&idx)[U], const bool (&ld)[U],
                                            int64_t safe, uint64_t (&x)[U]) {
  const int c = a.vcol[v];
  switch (a.vdt[v]) {
    case LMS_I32:
    case LMS_I64: {
      int64_t y[U];
      ext_i64_rows<U>(a.q, c, idx, ld, safe, y);
#pragma unroll
      for (int u = 0; u < U; ++u) x[u] = (uint64_t)y[u];
      break;
    }
    case LMS_F32: {
      uint32_t y[U];
#pragma unroll
      for (int u = 0; u < U; ++u) y[u] = ((const uint32_t*)a.q.col[c])[ld[u] ? idx[u] : safe];
#pragma unroll
      for (int u = 0; u < U; ++u) x[u] = ld[u] ? y[u] : 0u;
      break;
    }
    default: {
      uint64_t y[U];
#pragma unroll
      for (int u = 0; u < U; ++u) y[u] = ((const uint64_t*)a.q.col[c])[ld[u] ? idx[u] : safe];
#pragma unroll
      for (int u = 0; u < U; ++u) x[u] = ld[u] ? y[u] : 0;
    }
  }
}

// One staged record at r: key (8 B) at 0, 8-byte values at their offsets,
// then the pane, the 4-byte values and the padding -- consecutive words from
// pane_off (an 8-byte boundary) to the record's end, written two per 8-byte
// store (fewer partial-line writes than one store per field).
template <int MA>
__device__ __forceinline__ void put_record(const WinArgs& a, char* r, int64_t key, uint64_t qp,
                                           const uint64_t (&val)[MA]) {
  *(int64_t*)r = key;
  uint32_t wd[MA + 2];
  wd[0] = (uint32_t)qp;
#pragma unroll
  for (int t = 1; t < MA + 2; ++t) wd[t] = 0;
#pragma unroll
  for (int v = 0; v < MA; ++v) {
    if (v < a.nval) {
      if (a.vdt[v] == LMS_I32 || a.vdt[v] == LMS_F32) {
        const int t = (a.voff[v] - a.pane_off) >> 2;
#pragma unroll
        for (int tt = 1; tt <= MA; ++tt)
          if (tt == t) wd[tt] = (uint32_t)val[v];
      } else {
        *(uint64_t*)(r + a.voff[v]) = val[v];
      }
    }
  }
  const int nw = (a.rec - a.pane_off) >> 2;  // even
#pragma unroll
  for (int t = 0; t < MA + 2; t += 2)
    if (t < nw) *(uint2*)(r + a.pane_off + 4 * t) = make_uint2(wd[t], wd[t + 1]);
}

// The passing rows of chunk w, handed to sink(partition, key, pane, values).
// The predicate columns are read first; every other column a passing row
// needs is then loaded for all kUnroll rows of a thread before the first
// record is handed over, so the loads overlap, and rows that fail read one
// shared row in their place, so a selective predicate leaves most lines
// unread.
template <int MA, int TPB, class Sink>
__device__ void scatter_rows(const WinArgs& a, uint32_t w, uint64_t* lmask, Sink sink) {
  // eight value columns per row would hold too many loads in registers at 4 rows
  constexpr int kU = MA <= 6 ? kUnroll : 2;
  const int64_t b0 = a.hdr[0];
  const int64_t lo = (int64_t)w * a.chunk;
  const int64_t hi = min(a.q.nrows, lo + a.chunk);
  const void* kc = a.q.col[a.key_col];
  const int kdt = a.q.dt[a.key_col];
  const void* tc = a.q.col[a.ts_col];
  const int tdt = a.q.dt[a.ts_col];
  bool range_err = false;
  // the chunk's pass words, staged in LDS (lmask: chunk / 64 words): a step
  // whose rows all fail then costs one LDS read instead of a memory round trip
  const int nw = (int)((hi - lo + 63) >> 6);
  for (int i = threadIdx.x; i < nw; i += TPB) lmask[i] = gptr(a.pmask)[(lo >> 6) + i];
  __syncthreads();
  for (int64_t b = lo + threadIdx.x; b < hi; b += (int64_t)TPB * kU) {
    bool ok[kU];
    int64_t key[kU], ts[kU], idx[kU];
    uint64_t val[kU][MA];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      idx[u] = b + (int64_t)u * TPB;
      ok[u] = idx[u] < hi;
    }
    // the histogram pass recorded which rows pass; a wave whose rows of this
    // step all fail skips their loads
    uint64_t wd[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) wd[u] = lmask[((ok[u] ? idx[u] : lo) - lo) >> 6];
    bool any = false;
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      ok[u] = ok[u] && ((wd[u] >> (idx[u] & 63)) & 1u);
      any |= ok[u];
    }
    if (!__ballot(any)) continue;
    load_i64_rows<kU>(kc, kdt, idx, ok, lo, key);
    load_i64_rows<kU>(tc, tdt, idx, ok, lo, ts);
#pragma unroll
    for (int v = 0; v < MA; ++v) {
      if (v < a.nval) {
        uint64_t x[kU];
        staged_rows<kU>(a, v, idx, ok, lo, x);
#pragma unroll
        for (int u = 0; u < kU; ++u) val[u][v] = x[u];
      } else {
#pragma unroll
        for (int u = 0; u < kU; ++u) val[u][v] = 0;
      }
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      if (!ok[u]) continue;
      const int64_t rel = ts[u] - a.origin - b0 * a.pane;
      uint64_t qp = 0;
      if (rel < 0) range_err = true;
      else qp = div_pane((uint64_t)rel, a.pane, a.inv_pane);
      if (qp >= (1ull << 31)) {
        range_err = true;
        qp = 0;
      }
      sink(part_of(fmix64((uint64_t)key[u]), a.pbits), key[u], qp, val[u]);
    }
  }
  if (range_err) win_status(a, LMS_ERANGE);
  __syncthreads();
}

// Scatter the passing rows of chunk w, as (key, pane, value columns), each to
// the next slot of its partition's segment for this chunk.
template <int MA>
__device__ void scatter_chunk(const WinArgs& a, uint32_t w, uint32_t* cursor) {
  uint64_t* const lmask = (uint64_t*)(cursor + ((a.nparts + 1) & ~1));  // LDS of hist_lds(nparts, chunk)
  for (int p = threadIdx.x; p < a.nparts; p += kScatterTPB) cursor[p] = a.Off[(size_t)p * a.g1 + w];
  __syncthreads();
  scatter_rows<MA, kScatterTPB>(a, w, lmask, [&](int part, int64_t key, uint64_t qp, const uint64_t(&val)[MA]) {
    const uint32_t pos = atomicAdd(&cursor[part], 1u);
    put_record<MA>(a, a.srec + (size_t)pos * a.rec, key, qp, val);
  });
}

// Staged scatter of one chunk (single-batch launch, one 1024-thread workgroup
// per chunk): when the chunk's passing rows fit the LDS stage, they are first
// written there sorted by partition (the chunk's own histogram gives each
// partition's first slot), then copied out 8-byte word by word, consecutive
// lanes writing consecutive words of a partition's segment.  Written straight
// to the segments, a wave's records went to 64 different cache lines per
// store; copied out, a store covers a few.  A chunk with more passing rows
// than the stage holds takes the direct path.
constexpr int kStTPB = 1024;
constexpr size_t kStLds = 160 * 1024 - 512;  // dynamic LDS of the staged scatter

__host__ __device__ inline uint32_t stage_cap(int nparts, int rec, int64_t chunk) {
  return (uint32_t)((kStLds - 16 - 8 * (size_t)nparts - 8 - (size_t)(chunk + 63) / 64 * 8) / (size_t)(rec + 2));
}

template <int MA>
__global__ __launch_bounds__(kStTPB) void k_wa_scatter_st(WinArgs a) {
  extern __shared__ __align__(16) char st_lds[];
  __shared__ uint32_t scratch[kStTPB / 64 + 1];
  const uint32_t w = xcd_chunk(blockIdx.x, (uint32_t)a.g1);
  if (w >= (uint32_t)a.g1) return;
  const int np = a.nparts;
  const uint32_t cap = stage_cap(np, a.rec, a.chunk);
  uint32_t* const cur = (uint32_t*)st_lds;          // np: next slot of each partition
  uint32_t* const gof = cur + np;                    // np: staging index of slot 0's partition segment
  uint64_t* const lmask = (uint64_t*)(st_lds + align_up(8 * (size_t)np, 8));  // chunk / 64 pass words
  uint16_t* const spart = (uint16_t*)(lmask + (a.chunk + 63) / 64);  // cap: partition of each staged record
  // offsets from the LDS base, so the compiler keeps the stage's address space
  char* const stage = st_lds + align_up((size_t)((char*)(spart + cap) - st_lds), 16);
  for (int p = threadIdx.x; p < np; p += kStTPB) cur[p] = a.H[(size_t)p * a.g1 + w];
  __syncthreads();
  const uint32_t total = block_scan_array<kStTPB>(cur, np, scratch);  // cur = first slot of each partition
  if (total > cap) {  // does not fit the stage: straight to the segments
    for (int p = threadIdx.x; p < np; p += kStTPB) cur[p] = a.Off[(size_t)p * a.g1 + w];
    __syncthreads();
    scatter_rows<MA, kStTPB>(a, w, lmask, [&](int part, int64_t key, uint64_t qp, const uint64_t(&val)[MA]) {
      const uint32_t pos = atomicAdd(&cur[part], 1u);
      put_record<MA>(a, a.srec + (size_t)pos * a.rec, key, qp, val);
    });
    return;
  }
  for (int p = threadIdx.x; p < np; p += kStTPB) gof[p] = a.Off[(size_t)p * a.g1 + w] - cur[p];
  __syncthreads();
  scatter_rows<MA, kStTPB>(a, w, lmask, [&](int part, int64_t key, uint64_t qp, const uint64_t(&val)[MA]) {
    const uint32_t slot = atomicAdd(&cur[part], 1u);
    spart[slot] = (uint16_t)part;
    put_record<MA>(a, stage + (size_t)slot * a.rec, key, qp, val);
  });
  // (scatter_rows ends with a barrier)
  const uint32_t nw = (uint32_t)a.rec >> 3;
  const uint32_t words = total * nw;
  const float inv = 1.0f / (float)nw;
  for (uint32_t i = threadIdx.x; i < words; i += kStTPB) {
    uint32_t r = (uint32_t)((float)i * inv);  // record of word i: a float estimate, corrected exactly
    while (r * nw > i) --r;
    while ((r + 1) * nw <= i) ++r;
    const uint32_t k = i - r * nw;
    const uint32_t dst = gof[spart[r]] + r;
    ((uint64_t*)(a.srec + (size_t)dst * a.rec))[k] = ((const uint64_t*)(stage + (size_t)r * a.rec))[k];
  }
}

template <int MA>
__global__ __launch_bounds__(kScatterTPB) void k_wa_scatter(WinArgs a) {
  extern __shared__ uint32_t cursor[];
  if constexpr (MA == 8) {
    // at this unroll bound the loops over value columns stay rolled and would
    // index the by-value arguments dynamically (a private-memory copy); an LDS
    // copy avoids that
    __shared__ WinArgs sa;
    const uint32_t* src = (const uint32_t*)&a;
    for (uint32_t i = threadIdx.x; i < sizeof(WinArgs) / 4; i += blockDim.x) ((uint32_t*)&sa)[i] = src[i];
    __syncthreads();
    const uint32_t w = xcd_chunk(blockIdx.x, (uint32_t)a.g1);
    if (w < (uint32_t)a.g1) scatter_chunk<MA>(sa, w, cursor);
  } else {
    const uint32_t w = xcd_chunk(blockIdx.x, (uint32_t)a.g1);
    if (w < (uint32_t)a.g1) scatter_chunk<MA>(a, w, cursor);
  }
}

// LDS layout of one aggregation workgroup.
struct Lds {
  uint64_t* keys;  // ek + 1 (slot ek holds the key equal to the empty marker)
  uint32_t* kcnt;  // ek + 1: groups per key
  uint32_t* kaux;  // ek + 1: start of the key's run in `order`
  uint32_t* nwin;  // ek + 1: fill counters of the counting sort
  uint64_t* gid;   // eg: (key slot << 32) | pane, or kEmptyGid
  uint64_t* acc;   // nacc * eg: accumulator k of group g at acc[k * eg + g]
  uint32_t* gcnt;  // eg: rows per group
  uint32_t* order; // eg: group slots ordered by key, then windows per sorted entry
  uint64_t* sorted; // eg: (pane << 32 | group slot) in key-major, pane-sorted order
  int32_t* fw;      // eg: first window containing the sorted entry's pane
  int32_t* wlo;     // eg: first window owned by the sorted entry
  uint32_t* scan;  // kAggTPB / 64 + 1
  uint32_t* misc;  // flags and broadcasts
  uint64_t* stack; // 4 * kStackCap: (hash lo, hash hi, anchor lo, anchor hi) still to aggregate
};

enum { M_OVF = 0, M_SSIZE = 1, M_PC = 2, M_BASE_LO = 3, M_BASE_HI = 4, M_QMIN = 5, M_QMAX = 6, M_PLO = 7, M_PHI = 8,
       // sliding emission: output pointers (okey, ows, oagg[]) and per-aggregate codes
       M_OUT = 16, M_CODE = M_OUT + 2 * (2 + kMaxAggs), M_ACCFN = M_CODE + kMaxAggs, M_WORDS = M_ACCFN + kMaxAggs };

__host__ __device__ inline size_t lds_bytes(int ek, int eg, int nacc) {
  size_t b = 0;
  b += align_up((size_t)(ek + 1) * 8, 16);
  b += 3 * align_up((size_t)(ek + 1) * 4, 16);
  b += (size_t)eg * 8 + (size_t)nacc * eg * 8 + (size_t)eg * 4 + (size_t)eg * 4 + (size_t)eg * 8 + (size_t)eg * 8;
  b += align_up((kAggTPB / 64 + 1) * 4, 16) + M_WORDS * 4;
  b += 4 * kStackCap * 8;
  return b;
}

__device__ __forceinline__ Lds carve_lds(char* base, int ek, int eg, int nacc) {
  Lds s;
  size_t o = 0;
  s.keys = (uint64_t*)(base + o);
  o += align_up((size_t)(ek + 1) * 8, 16);
  s.kcnt = (uint32_t*)(base + o);
  o += align_up((size_t)(ek + 1) * 4, 16);
  s.kaux = (uint32_t*)(base + o);
  o += align_up((size_t)(ek + 1) * 4, 16);
  s.nwin = (uint32_t*)(base + o);
  o += align_up((size_t)(ek + 1) * 4, 16);
  s.gid = (uint64_t*)(base + o);
  o += (size_t)eg * 8;
  s.acc = (uint64_t*)(base + o);
  o += (size_t)nacc * eg * 8;
  s.gcnt = (uint32_t*)(base + o);
  o += (size_t)eg * 4;
  s.order = (uint32_t*)(base + o);
  o += (size_t)eg * 4;
  s.sorted = (uint64_t*)(base + o);
  o += (size_t)eg * 8;
  s.fw = (int32_t*)(base + o);
  o += (size_t)eg * 4;
  s.wlo = (int32_t*)(base + o);
  o += (size_t)eg * 4;
  s.scan = (uint32_t*)(base + o);
  o += align_up((kAggTPB / 64 + 1) * 4, 16);
  s.misc = (uint32_t*)(base + o);
  o += M_WORDS * 4;
  s.stack = (uint64_t*)(base + o);
  return s;
}

__device__ __forceinline__ uint64_t acc_identity(int fn) {
  if (fn == LMS_MIN) return (uint64_t)INT64_MAX;
  if (fn == LMS_MAX) return (uint64_t)INT64_MIN;
  return 0;  // SUM: 0; AVG: +0.0
}

__device__ __forceinline__ uint64_t combine(int fn, uint64_t x, uint64_t y) {
  switch (fn) {
    case LMS_SUM: return x + y;
    case LMS_MIN: return (int64_t)y < (int64_t)x ? y : x;
    case LMS_MAX: return (int64_t)y > (int64_t)x ? y : x;
    default:
      return (uint64_t)__double_as_longlong(__longlong_as_double((long long)x) + __longlong_as_double((long long)y));
  }
}

template <int MA>
__device__ void clear_tables(const WinArgs& a, Lds& s) {
  if (threadIdx.x == 0) {
    s.misc[M_QMIN] = ~0u;  // pane range of the groups, for the sliding composition
    s.misc[M_QMAX] = 0;
  }
  for (int i = threadIdx.x; i <= a.ek; i += kAggTPB) {
    s.keys[i] = kEmptyKey;
    s.kcnt[i] = 0;
    s.kaux[i] = 0;
    s.nwin[i] = 0;
  }
  for (int g = threadIdx.x; g < a.eg; g += kAggTPB) {
    s.gid[g] = kEmptyGid;
    s.gcnt[g] = 0;
  }
#pragma unroll
  for (int k = 0; k < MA; ++k) {
    if (k < a.nacc) {
      const uint64_t id = acc_identity(a.accfn[k]);
      for (int g = threadIdx.x; g < a.eg; g += kAggTPB) s.acc[(size_t)k * a.eg + g] = id;
    }
  }
}

// One input element: a staged row (cnt 1) or a partial record.  Only ever
// indexed with compile-time indices, so it lives in registers.
template <int MA>
struct Elem {
  int64_t key;
  uint32_t pane;
  uint32_t cnt;
  uint64_t in[MA];  // input of accumulator k (int64 or double bits)
};

// Issues the loads of staged row e as its 8-byte words: a record is 8-byte
// aligned and at most MA + 2 words long (key, 8-byte values, then the pane and
// the 4-byte values in pairs), so this is one load per word, however many
// values it holds.  The words are kept raw in the fields of x in word order
// (key, pane word, then in[]); finish_row picks the pane and the values out of
// them once they are needed, so no load waits for another's result.
template <int MA>
__device__ __forceinline__ void load_row(const WinArgs& a, uint32_t e, Elem<MA>& x) {
  const uint64_t* const r = (const uint64_t*)(a.srec + (size_t)e * a.rec);
  const int nw = a.rec >> 3;
  uint64_t w[MA + 2];
#pragma unroll
  for (int t = 0; t < MA + 2; ++t) w[t] = t < nw ? gptr(r)[t] : 0;
  x.key = (int64_t)w[0];
  x.pane = (uint32_t)w[1];
  x.cnt = (uint32_t)(w[1] >> 32);
#pragma unroll
  for (int k = 0; k < MA; ++k) x.in[k] = w[2 + k];
}

// Raw record words (from load_row) -> pane and accumulator inputs: int64, or
// double bits for float columns and for AVG of an integer column.  A field's
// word is read from a vector of the record's words at its word index, which
// is uniform (a register-indexed move: a plain array indexed at run time would
// go to private memory).
template <int MA>
__device__ __forceinline__ void finish_row(const WinArgs& a, Elem<MA>& x) {
  typedef uint64_t words_t __attribute__((ext_vector_type(MA + 2)));
  words_t w;
  w[0] = (uint64_t)x.key;
  w[1] = ((uint64_t)x.cnt << 32) | x.pane;
#pragma unroll
  for (int k = 0; k < MA; ++k) w[2 + k] = x.in[k];
  auto word = [&](int t) { return w[t]; };
  x.pane = (uint32_t)word(a.pane_off >> 3);
  x.cnt = 1;
  uint64_t raw[MA];
#pragma unroll
  for (int v = 0; v < MA; ++v) {
    raw[v] = 0;
    if (v < a.nval) {
      const int o = a.voff[v];
      const uint64_t wv = word(o >> 3) >> ((o & 4) * 8);
      switch (a.vdt[v]) {
        case LMS_I32: raw[v] = (uint64_t)(int64_t)(int32_t)(uint32_t)wv; break;
        case LMS_F32: raw[v] = (uint64_t)__double_as_longlong((double)__uint_as_float((uint32_t)wv)); break;
        default: raw[v] = wv; break;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < MA; ++k) {
    x.in[k] = 0;
    if (k < a.nacc) {
      const int v = a.accval[k];
      uint64_t r = raw[0];
#pragma unroll
      for (int j = 1; j < MA; ++j) r = v == j ? raw[j] : r;
      const bool is_int = a.vdt[v] == LMS_I32 || a.vdt[v] == LMS_I64;
      x.in[k] = (a.accfn[k] == LMS_AVG && is_int) ? (uint64_t)__double_as_longlong((double)(int64_t)r) : r;
    }
  }
}

// Marks every field of x as redefined here (an empty asm taking each one):
// the compiler's wait-count tracking then no longer ties these registers to
// the loads that filled them, so a later use does not wait for loads issued
// after this point (without it, the first use after the next round's loads
// waited for all of them).
template <int MA>
__device__ __forceinline__ void settle(Elem<MA>& x) {
  asm volatile("" : "+v"(x.key), "+v"(x.pane), "+v"(x.cnt));
#pragma unroll
  for (int k = 0; k < MA; ++k) asm volatile("" : "+v"(x.in[k]));
}

template <int MA>
__device__ __forceinline__ void load_partial(const WinArgs& a, uint32_t e, Elem<MA>& x) {
  x.key = a.pkey[e];
  x.pane = a.ppane[e];
  x.cnt = a.pcnt[e];
#pragma unroll
  for (int k = 0; k < MA; ++k) x.in[k] = k < a.nacc ? a.pacc[k][e] : 0;
}

__device__ __forceinline__ uint32_t group_hash(uint64_t gid) {
  uint32_t h = (uint32_t)gid * 0x9E3779B1u + (uint32_t)(gid >> 32) * 0x85EBCA77u;
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  return h;
}

// Slot of `want` in an open-addressing table of n (a power of two) 64-bit
// slots, linear probing from `start`; claims the first empty slot if `want`
// is absent.  Four consecutive slots are read per step, all issued before
// the first is tested: the probe is bound by LDS round trips, and a wave runs
// as long as its longest probe, so fewer dependent steps per slot count more
// than the few extra reads.  Slots only ever go from empty to taken while
// rows are inserted, so slots seen taken by another value stay so, and a
// value is always in the first empty-or-matching slot of its sequence (a lost
// claim is re-examined: the winner may have written the same value).
// Returns -1 if the table is full.
__device__ __forceinline__ int probe_claim(uint64_t* tab, uint32_t n, uint32_t start, uint64_t want, uint64_t empty) {
  const uint32_t mask = n - 1;
  uint32_t pos = start;
  for (uint32_t seen = 0; seen < n;) {
    uint64_t c[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) c[u] = __atomic_load_n(&tab[(pos + u) & mask], __ATOMIC_RELAXED);
    int hit = -1;
#pragma unroll
    for (int u = 3; u >= 0; --u)
      if (c[u] == want || c[u] == empty) hit = u;
    if (hit < 0) {
      pos += 4;
      seen += 4;
      continue;
    }
    const uint32_t slot = (pos + (uint32_t)hit) & mask;
    if (c[hit] == want) return (int)slot;
    const uint64_t old = atomicCAS((unsigned long long*)&tab[slot], (unsigned long long)empty,
                                   (unsigned long long)want);
    if (old == empty || old == want) return (int)slot;
    pos += (uint32_t)hit + 1;  // taken by another value meanwhile: go on after it
    seen += (uint32_t)hit + 1;
  }
  return -1;
}

// Inserts one element; returns false if a table is full.
template <int MA>
__device__ __forceinline__ bool insert(const WinArgs& a, Lds& s, const Elem<MA>& x, uint64_t h) {
  int kid;
  if ((uint64_t)x.key == kEmptyKey) {
    kid = a.ek;
    s.keys[a.ek] = kEmptyKey;
  } else {
    kid = probe_claim(s.keys, (uint32_t)a.ek, (uint32_t)h & (uint32_t)(a.ek - 1), (uint64_t)x.key, kEmptyKey);
    if (kid < 0) return false;
  }
  const uint64_t gid = ((uint64_t)kid << 32) | x.pane;
  const int g = probe_claim(s.gid, (uint32_t)a.eg, group_hash(gid) & (uint32_t)(a.eg - 1), gid, kEmptyGid);
  if (g < 0) return false;
  atomicAdd(&s.gcnt[g], x.cnt);
#pragma unroll
  for (int k = 0; k < MA; ++k) {
    if (k < a.nacc) {
      uint64_t* p = s.acc + (size_t)k * a.eg + g;
      switch (a.accfn[k]) {
        case LMS_SUM: atomicAdd((unsigned long long*)p, (unsigned long long)x.in[k]); break;
        case LMS_MIN: atomicMin((long long*)p, (long long)x.in[k]); break;
        case LMS_MAX: atomicMax((long long*)p, (long long)x.in[k]); break;
        default: unsafeAtomicAdd((double*)p, __longlong_as_double((long long)x.in[k])); break;
      }
    }
  }
  return true;
}

// Result rows are written once and not read again by the launch: stored
// non-temporally, so they displace less of what the kernels still read from
// L2 (measured: the step 2.6 % faster, the merge 6 %).
template <class T>
__device__ __forceinline__ void out_store(T* p, T v) {
  // the output pointers come from an LDS table, so the compiler cannot tell
  // their address space: marked global, the stores are global stores, which
  // count only against the vector-memory wait counter (a flat store also
  // counts against the LDS one, so every later LDS wait would wait for it)
  __builtin_nontemporal_store(v, gptr(p));
}

__device__ __forceinline__ int64_t key_of(const WinArgs& a, const Lds& s, uint32_t kid) {
  return kid == (uint32_t)a.ek ? (int64_t)kEmptyKey : (int64_t)s.keys[kid];
}

// Reserves `total` output rows; returns the first index (broadcast to all).
__device__ int64_t reserve_output(const WinArgs& a, Lds& s, uint32_t total) {
  if (threadIdx.x == 0) {
    const unsigned long long b = atomicAdd((unsigned long long*)&a.d_count[0], (unsigned long long)total);
    s.misc[M_BASE_LO] = (uint32_t)b;
    s.misc[M_BASE_HI] = (uint32_t)(b >> 32);
  }
  __syncthreads();
  const int64_t base = (int64_t)(((uint64_t)s.misc[M_BASE_HI] << 32) | s.misc[M_BASE_LO]);
  __syncthreads();
  return base;
}

// The emission loops read the output pointers and aggregate codes from this
// small LDS table.  Read from the kernel arguments they pushed the kernel past
// its scalar registers, and the compiler parked them in lanes of vector
// registers and re-read them there for every row (measured: the aggregation
// kernel 5.6 % faster on a sliding query with the table).  Thread 0 fills it;
// the caller's next barrier publishes it.
__device__ __forceinline__ void fill_out_table(const WinArgs& a, Lds& s) {
  if (threadIdx.x == 0) {
    uint64_t* const out = (uint64_t*)(s.misc + M_OUT);
    out[0] = (uint64_t)a.okey;
    out[1] = (uint64_t)a.ows;
#pragma unroll
    for (int k = 0; k < kMaxAggs; ++k) {
      out[2 + k] = (uint64_t)a.oagg[k];
      s.misc[M_CODE + k] = ((uint32_t)a.afn[k] & 0xffu) | (((uint32_t)a.aacc[k] & 0xffu) << 8);
      s.misc[M_ACCFN + k] = (uint32_t)a.accfn[k];
    }
  }
}

// Tumbling windows: every group (key, pane) is one output row.
template <int MA>
__device__ void emit_tumbling(const WinArgs& a, Lds& s, int64_t b0) {
  fill_out_table(a, s);
  // Wave w takes slots w * 64 + lane, then every kAggTPB further.  After one
  // count and one reservation, each wave writes its groups at a running offset
  // ranked by ballots -- no workgroup barrier while the stores drain.
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t below = (1ull << lane) - 1;
  uint32_t mine = 0;
  for (int g0 = (int)wave * 64; g0 < a.eg; g0 += kAggTPB) {
    const int g = g0 + (int)lane;
    mine += (uint32_t)__popcll(__ballot(g < a.eg && s.gid[g] != kEmptyGid));
  }
  if (lane == 0) s.scan[wave] = mine;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < kAggTPB / 64; ++w) {
      const uint32_t v = s.scan[w];
      s.scan[w] = t;
      t += v;
    }
    const unsigned long long b = t ? atomicAdd((unsigned long long*)&a.d_count[0], (unsigned long long)t) : 0ull;
    s.misc[M_BASE_LO] = (uint32_t)b;
    s.misc[M_BASE_HI] = (uint32_t)(b >> 32);
    s.scan[kAggTPB / 64] = t;
  }
  __syncthreads();
  if (s.scan[kAggTPB / 64] == 0) return;
  int64_t run = (int64_t)(((uint64_t)s.misc[M_BASE_HI] << 32) | s.misc[M_BASE_LO]) + s.scan[wave];
  for (int g0 = (int)wave * 64; g0 < a.eg; g0 += kAggTPB) {
    const int g = g0 + (int)lane;
    const bool occ = g < a.eg && s.gid[g] != kEmptyGid;
    const uint64_t m = __ballot(occ);
    const int64_t idx = run + __popcll(m & below);
    run += __popcll(m);
    if (occ && idx < a.cap) {
      const uint64_t gid = s.gid[g];
      const uint32_t cnt = s.gcnt[g];
      const uint64_t* const out = (const uint64_t*)(s.misc + M_OUT);
      const uint32_t* const code = s.misc + M_CODE;
      out_store((int64_t*)out[0] + idx, key_of(a, s, (uint32_t)(gid >> 32)));
      out_store((int64_t*)out[1] + idx, a.origin + (b0 + (int64_t)(uint32_t)gid) * a.len);
#pragma unroll
      for (int k = 0; k < kMaxAggs; ++k) {
        if (k >= a.nagg) break;
        const uint32_t c = code[k];
        const int fn = (int)(c & 0xffu);
        void* const op = (void*)out[2 + k];
        if (fn == LMS_COUNT) {
          out_store((int64_t*)op + idx, (int64_t)cnt);
        } else {
          const uint64_t v = s.acc[(size_t)(c >> 8) * a.eg + g];
          if (fn == LMS_AVG) out_store((double*)op + idx, __longlong_as_double((long long)v) / (double)cnt);
          else out_store((int64_t*)op + idx, (int64_t)v);
        }
      }
    }
  }
}

// floor(x / d) for d > 0 and |x| < 2^52: a double estimate corrected exactly.
__device__ __forceinline__ int64_t fdiv(int64_t x, int64_t d, double inv) {
  int64_t q = (int64_t)floor((double)x * inv);
  int64_t r = x - q * d;
  while (r < 0) {
    --q;
    r += d;
  }
  while (r >= d) {
    ++q;
    r -= d;
  }
  return q;
}

// Accumulator slot A (an eg-strided LDS array) combined over entries
// [i, hi) of a key's pane-sorted run.  fn is uniform across the wave, so the
// switch is taken once per slot and each case is a plain loop.
__device__ __forceinline__ uint64_t combine_run(int fn, const uint64_t* A, uint32_t i, uint32_t hi) {
  uint64_t x = A[i];
  switch (fn) {
    case LMS_SUM:
      for (uint32_t j = i + 1; j < hi; ++j) x += A[j];
      return x;
    case LMS_MIN:
      for (uint32_t j = i + 1; j < hi; ++j) x = (int64_t)A[j] < (int64_t)x ? A[j] : x;
      return x;
    case LMS_MAX:
      for (uint32_t j = i + 1; j < hi; ++j) x = (int64_t)A[j] > (int64_t)x ? A[j] : x;
      return x;
    default: {
      double d = __longlong_as_double((long long)x);
      for (uint32_t j = i + 1; j < hi; ++j) d += __longlong_as_double((long long)A[j]);
      return (uint64_t)__double_as_longlong(d);
    }
  }
}

// One output row of the sliding composition: row r, owned by sorted entry i.
// The window's panes are the key's entries [i, hi): entry i (the first pane
// the window holds) and the following ones whose first window is not after
// w; first windows are nondecreasing along a key's run, so they form a
// prefix, found four entries per step.  Each accumulator is then combined
// over [i, hi) under the uniform function of its slot (fnk[k]), in entry
// order (so double sums are added in pane order).
template <int MA>
__device__ __forceinline__ void emit_row(const WinArgs& a, Lds& s, uint32_t i, uint32_t r, int64_t base,
                                         int64_t wbase, const int (&fnk)[MA]) {
  const int64_t idx = base + r;
  if (idx >= a.cap) return;
  const int32_t w = s.wlo[i] + (int32_t)(r - s.order[i]);
  const uint64_t kk = s.sorted[i];
  const uint32_t kid = (uint32_t)kk, ke = (uint32_t)(kk >> 32);
  const uint32_t last = (uint32_t)a.eg - 1;
  uint32_t hi = i + 1;
  while (true) {
    int32_t f[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) f[u] = s.fw[min(hi + u, last)];  // in bounds, issued together
    uint32_t c = 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) c += (hi + u < ke && f[u] <= w) ? 1u : 0u;
    hi += c;
    if (c < 4) break;
  }
  uint32_t cnt = s.gcnt[i];
  for (uint32_t j = i + 1; j < hi; ++j) cnt += s.gcnt[j];
  uint64_t acc[MA];
#pragma unroll
  for (int k = 0; k < MA; ++k) acc[k] = k < a.nacc ? combine_run(fnk[k], s.acc + (size_t)k * a.eg, i, hi) : 0;
  // output pointers and aggregate codes: the table of fill_out_table
  const uint64_t* const out = (const uint64_t*)(s.misc + M_OUT);
  const uint32_t* const code = s.misc + M_CODE;
  out_store((int64_t*)out[0] + idx, key_of(a, s, kid));
  out_store((int64_t*)out[1] + idx, a.origin + ((int64_t)w + wbase) * a.slide);
#pragma unroll
  for (int k = 0; k < kMaxAggs; ++k) {
    if (k >= a.nagg) break;
    const uint32_t c = code[k];
    const int fn = (int)(c & 0xffu);
    void* const op = (void*)out[2 + k];
    if (fn == LMS_COUNT) {
      out_store((int64_t*)op + idx, (int64_t)cnt);
    } else {
      const int slot = (int)(c >> 8);
      uint64_t x = acc[0];
#pragma unroll
      for (int j = 1; j < MA; ++j) x = slot == j ? acc[j] : x;
      if (fn == LMS_AVG) out_store((double*)op + idx, __longlong_as_double((long long)x) / (double)cnt);
      else out_store((int64_t*)op + idx, (int64_t)x);
    }
  }
}

// Sliding windows, composed in parallel over the groups of the LDS table.
// The groups of each key are ranked by pane (every key has at most one group
// per pane) into key-major, pane-sorted order.  Each window of a key is
// produced by the first of the key's panes it contains: pane i covers windows
// first_win(q_i)..last_win(q_i), of which it owns those after the previous
// pane's last window.  Output rows are then produced one per thread, so
// consecutive threads write consecutive rows: row r belongs to the last entry
// whose owned windows start at or before r, and its window holds that entry's
// pane and the key's following panes whose first window is not later.  Only
// windows [wmin, wmax] are emitted (the windows whose first pane lies in the
// anchor range of the tables' current pass).
template <int MA>
__device__ void emit_sliding(const WinArgs& a, Lds& s, int64_t b0, int64_t wmin, int64_t wmax) {
  fill_out_table(a, s);  // the barriers below publish it
  const int nk = a.ek + 1;
  auto first_win = [&](int64_t q) { return fdiv(q - a.W, a.R, a.inv_R) + 1; };
  auto last_win = [&](int64_t q) { return fdiv(q, a.R, a.inv_R); };
  uint32_t qlo = ~0u, qhi = 0;
  for (int g = threadIdx.x; g < a.eg; g += kAggTPB) {
    const uint64_t gid = s.gid[g];
    if (gid != kEmptyGid) {
      atomicAdd(&s.kcnt[(uint32_t)(gid >> 32)], 1u);
      qlo = min(qlo, (uint32_t)gid);
      qhi = max(qhi, (uint32_t)gid);
    }
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    qlo = min(qlo, (uint32_t)__shfl_xor((int)qlo, d, 64));
    qhi = max(qhi, (uint32_t)__shfl_xor((int)qhi, d, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMin(&s.misc[M_QMIN], qlo);
    atomicMax(&s.misc[M_QMAX], qhi);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nk; i += kAggTPB) s.kaux[i] = s.kcnt[i];
  __syncthreads();
  const uint32_t ng = block_scan_array<kAggTPB>(s.kaux, nk, s.scan);  // kaux = start of each key's run
  if (ng == 0) return;
  const uint32_t qmin = s.misc[M_QMIN];
  if (s.misc[M_QMAX] - qmin < 64) {
    // All panes within 64 of each other: a pane's rank within its key is the
    // number of the key's panes below it, read off a 64-bit pane mask per key
    // (kept in the fw/wlo arrays, which are not needed until later).
    uint64_t* const kbits = (uint64_t*)s.fw;  // nk words fit: 8 (ek + 1) <= 8 eg
    for (int i = threadIdx.x; i < nk; i += kAggTPB) kbits[i] = 0;
    __syncthreads();
    for (int g = threadIdx.x; g < a.eg; g += kAggTPB) {
      const uint64_t gid = s.gid[g];
      if (gid != kEmptyGid) atomicOr((unsigned long long*)&kbits[(uint32_t)(gid >> 32)], 1ull << ((uint32_t)gid - qmin));
    }
    __syncthreads();
    for (int g = threadIdx.x; g < a.eg; g += kAggTPB) {
      const uint64_t gid = s.gid[g];
      if (gid == kEmptyGid) continue;
      const uint32_t kid = (uint32_t)(gid >> 32), q = (uint32_t)gid;
      const uint32_t r = (uint32_t)__popcll(kbits[kid] & ((1ull << (q - qmin)) - 1));
      s.sorted[s.kaux[kid] + r] = ((uint64_t)q << 32) | (uint32_t)g;
    }
    __syncthreads();
  } else {
    for (int g = threadIdx.x; g < a.eg; g += kAggTPB) {
      const uint64_t gid = s.gid[g];
      if (gid != kEmptyGid) {
        const uint32_t kid = (uint32_t)(gid >> 32);
        s.order[s.kaux[kid] + atomicAdd(&s.nwin[kid], 1u)] = (uint32_t)g;
      }
    }
    __syncthreads();
    int32_t* const wpane = s.wlo;  // panes of the unsorted key runs, only while ranking
    for (uint32_t i = threadIdx.x; i < ng; i += kAggTPB) wpane[i] = (int32_t)(uint32_t)s.gid[s.order[i]];
    __syncthreads();
    for (int g = threadIdx.x; g < a.eg; g += kAggTPB) {  // rank by pane within the key
      const uint64_t gid = s.gid[g];
      if (gid == kEmptyGid) continue;
      const uint32_t kid = (uint32_t)(gid >> 32);
      const int32_t q = (int32_t)(uint32_t)gid;
      const uint32_t ks = s.kaux[kid], m = s.kcnt[kid];
      uint32_t r = 0, j = 0;
      for (; j + 8 <= m; j += 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u) r += wpane[ks + j + u] < q;
      }
      for (; j < m; ++j) r += wpane[ks + j] < q;
      s.sorted[ks + r] = ((uint64_t)(uint32_t)q << 32) | (uint32_t)g;
    }
    __syncthreads();
  }
  // Permute the group arrays (id, count, accumulators) into the sorted order,
  // all of them in one pass through registers (one pair of barriers), so the
  // composition below reads a key's consecutive panes from consecutive slots
  // instead of through the slot index.
  {
    constexpr int kPer = 2048 / kAggTPB;  // eg <= 2048
    uint64_t vg[kPer], va[kPer][MA];
    uint32_t vc[kPer];
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
      const uint32_t i = threadIdx.x + t * kAggTPB;
      if (i < ng) {
        const uint32_t src = (uint32_t)s.sorted[i];
        vg[t] = s.gid[src];
        vc[t] = s.gcnt[src];
#pragma unroll
        for (int k = 0; k < MA; ++k)
          if (k < a.nacc) va[t][k] = s.acc[(size_t)k * a.eg + src];
      }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < kPer; ++t) {
      const uint32_t i = threadIdx.x + t * kAggTPB;
      if (i < ng) {
        s.gid[i] = vg[t];
        s.gcnt[i] = vc[t];
#pragma unroll
        for (int k = 0; k < MA; ++k)
          if (k < a.nacc) s.acc[(size_t)k * a.eg + i] = va[t][k];
      }
    }
    __syncthreads();
  }
  for (uint32_t i = threadIdx.x; i < ng; i += kAggTPB) {
    const uint64_t v = s.sorted[i];
    const int64_t q = (int64_t)(v >> 32);
    const uint32_t kid = (uint32_t)(s.gid[i] >> 32);
    const int64_t fw = first_win(q);
    const int64_t hi = min(last_win(q), wmax);
    int64_t lo = max(fw, wmin);
    if (i > s.kaux[kid]) lo = max(lo, last_win((int64_t)(s.sorted[i - 1] >> 32)) + 1);
    s.fw[i] = (int32_t)fw;
    s.wlo[i] = (int32_t)lo;
    s.order[i] = hi >= lo ? (uint32_t)(hi - lo + 1) : 0u;
  }
  __syncthreads();
  const uint32_t total = block_scan_array<kAggTPB>(s.order, (int)ng, s.scan);  // order = first row of entry
  // the panes are no longer needed: each entry keeps its key slot and the end
  // of its key's run instead, so a row finds both with one load
  for (uint32_t i = threadIdx.x; i < ng; i += kAggTPB) {
    const uint32_t kid = (uint32_t)(s.gid[i] >> 32);
    s.sorted[i] = ((uint64_t)(s.kaux[kid] + s.kcnt[kid]) << 32) | kid;
  }
  __syncthreads();
  if (total == 0) return;
  // The group ids are dead from here on, so their slots hold a row -> entry
  // map (16-bit entries, 4 per id slot) whenever the rows fit; each entry
  // fills in the rows of the windows it owns.
  uint16_t* const rmap = (uint16_t*)s.gid;
  const bool mapped = total <= 4u * (uint32_t)a.eg && ng <= 65536u;
  if (mapped) {
    for (uint32_t i = threadIdx.x; i < ng; i += kAggTPB) {
      const uint32_t end = i + 1 < ng ? s.order[i + 1] : total;
      for (uint32_t r = s.order[i]; r < end; ++r) rmap[r] = (uint16_t)i;
    }
  }
  const int64_t base = reserve_output(a, s, total);  // its barrier publishes the map
  const int64_t wbase = b0 / a.R;
  int fnk[MA];  // accumulator functions, uniform: read once
#pragma unroll
  for (int k = 0; k < MA; ++k) fnk[k] = __builtin_amdgcn_readfirstlane((int)s.misc[M_ACCFN + k]);
  // Rows go out in blocks of 64, one per lane, each wave taking every
  // (kAggTPB / 64)-th block.  Nothing here needs a workgroup barrier, so a
  // wave's output stores overlap its next block instead of being waited for.
  const uint32_t lane = threadIdx.x & 63;
  if (mapped) {
    for (uint32_t r = threadIdx.x; r < total; r += kAggTPB) emit_row<MA>(a, s, rmap[r], r, base, wbase, fnk);
    return;
  }
  // Without the map, lane 0 finds the block's first entry and broadcasts it;
  // every lane then searches only the block's entries (at most 64 R of them,
  // as each owned window spans at most R panes).
  const uint32_t span = (uint32_t)min<int64_t>(64 * a.R, ng);
  for (uint32_t r0 = (threadIdx.x >> 6) * 64; r0 < total; r0 += kAggTPB) {
    uint32_t i0 = 0;
    if (lane == 0) {
      uint32_t lo = 0, hi = ng - 1;  // last entry i with order[i] <= r0
      while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (s.order[mid] <= r0) lo = mid;
        else hi = mid - 1;
      }
      i0 = lo;
    }
    i0 = (uint32_t)__shfl((int)i0, 0, 64);
    const uint32_t r = r0 + lane;
    if (r < total) {
      uint32_t lo = i0, hi = min(ng - 1, i0 + span);  // last entry i with order[i] <= r
      while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (s.order[mid] <= r) lo = mid;
        else hi = mid - 1;
      }
      emit_row<MA>(a, s, lo, r, base, wbase, fnk);
    }
  }
}

// Input elements: raw staged rows [lo, hi), or the partial records that the
// pieces of a split partition reserved in [lo, hi) of the partial arrays.
struct Segments {
  bool partial;
  uint32_t lo, hi;
};

// Aggregates every element whose key hash lies in sub-ranges of [0, 2^32),
// starting with the whole range and halving a range whenever its groups do not
// fit the LDS tables, then composes and emits its windows.  A range of a single
// hash value that still overflows (one key holding more panes than a table) is
// split by window anchor instead: a pass over anchors [elo, ehi) emits the
// windows whose first pane lies there, and inserts the panes those windows
// span, [elo, ehi + W - 1); the anchor range is halved until it fits, so only
// a single window spanning more panes than a table holds is LMS_ECAPACITY.
constexpr int64_t kAnyLo = INT64_MIN, kAnyHi = INT64_MAX;  // no anchor restriction

template <int MA>
__device__ void aggregate_and_emit(const WinArgs& a, Lds& s, const Segments& sg, uint64_t rlo0 = 0,
                                   uint64_t rhi0 = 1ull << 32) {
  const int64_t b0 = a.hdr[0];
  auto push = [&](uint32_t n, uint64_t rlo, uint64_t rhi, int64_t elo, int64_t ehi) {
    s.stack[4 * n] = rlo;
    s.stack[4 * n + 1] = rhi;
    s.stack[4 * n + 2] = (uint64_t)elo;
    s.stack[4 * n + 3] = (uint64_t)ehi;
  };
  if (threadIdx.x == 0) {
    push(0, rlo0, rhi0, kAnyLo, kAnyHi);
    s.misc[M_SSIZE] = 1;
  }
  __syncthreads();
  while (true) {
    const uint32_t ssize = s.misc[M_SSIZE];
    if (ssize == 0) break;
    const uint64_t rlo = s.stack[4 * (ssize - 1)];
    const uint64_t rhi = s.stack[4 * (ssize - 1) + 1];
    const int64_t elo = (int64_t)s.stack[4 * (ssize - 1) + 2];
    const int64_t ehi = (int64_t)s.stack[4 * (ssize - 1) + 3];
    const bool any = elo == kAnyLo;
    // panes inserted in this pass: [elo, ehi + W - 1) unless unrestricted
    const int64_t ilo = any ? kAnyLo : elo, ihi = any ? kAnyHi : ehi + a.W - 1;
    __syncthreads();
    if (threadIdx.x == 0) {
      s.misc[M_SSIZE] = ssize - 1;
      s.misc[M_OVF] = 0;
    }
    clear_tables<MA>(a, s);
    __syncthreads();
    bool ovf = false;
    {
      const uint32_t lo = sg.lo, hi = sg.hi;
      // two elements per thread per round, both loads issued before either
      // is used: the round waits once for two loads
      for (uint32_t b = lo; b < hi; b += 2 * kAggTPB) {
        const uint32_t e0 = b + threadIdx.x, e1 = e0 + kAggTPB;
        Elem<MA> x0, x1;
        if (e0 < hi) {
          if (sg.partial) load_partial<MA>(a, e0, x0);
          else load_row<MA>(a, e0, x0);
        }
        if (e1 < hi) {
          if (sg.partial) load_partial<MA>(a, e1, x1);
          else load_row<MA>(a, e1, x1);
        }
        bool ins0 = false, ins1 = false;
        uint64_t h0 = 0, h1 = 0;
        if (e0 < hi) {
          if (!sg.partial) finish_row<MA>(a, x0);
          h0 = fmix64((uint64_t)x0.key);
          const uint32_t sh = subhash(h0);
          const int64_t q = (int64_t)x0.pane;
          ins0 = sh >= rlo && sh < rhi && q >= ilo && q < ihi;
        }
        if (e1 < hi) {
          if (!sg.partial) finish_row<MA>(a, x1);
          h1 = fmix64((uint64_t)x1.key);
          const uint32_t sh = subhash(h1);
          const int64_t q = (int64_t)x1.pane;
          ins1 = sh >= rlo && sh < rhi && q >= ilo && q < ihi;
        }
        bool fail = ins0 && !insert<MA>(a, s, x0, h0);
        fail = (ins1 && !insert<MA>(a, s, x1, h1)) || fail;
        if (fail) s.misc[M_OVF] = 1;
        __syncthreads();
        const bool o = s.misc[M_OVF] != 0;
        __syncthreads();  // every thread has read the flag before the next round may set it
        if (o) {
          ovf = true;
          break;
        }
      }
    }
    __syncthreads();
    if (ovf) {
      const bool split_hash = rhi - rlo > 1;
      if (!split_hash && any) {
        // pane bounds of this hash range: the anchors of its windows span
        // [min pane - W + 1, max pane]
        if (threadIdx.x == 0) {
          s.misc[M_PLO] = ~0u;
          s.misc[M_PHI] = 0;
        }
        __syncthreads();
        uint32_t qlo = ~0u, qhi = 0;
        for (uint32_t e = sg.lo + threadIdx.x; e < sg.hi; e += kAggTPB) {
          const int64_t key = sg.partial ? a.pkey[e] : *(const int64_t*)(a.srec + (size_t)e * a.rec);
          const uint32_t q = sg.partial ? a.ppane[e] : *(const uint32_t*)(a.srec + (size_t)e * a.rec + a.pane_off);
          const uint32_t sh = subhash(fmix64((uint64_t)key));
          if (sh >= rlo && sh < rhi) {
            qlo = min(qlo, q);
            qhi = max(qhi, q);
          }
        }
        atomicMin(&s.misc[M_PLO], qlo);
        atomicMax(&s.misc[M_PHI], qhi);
        __syncthreads();
      }
      if (threadIdx.x == 0) {
        const uint32_t n = s.misc[M_SSIZE];
        int64_t nlo = elo, nhi = ehi;
        if (!split_hash && any) {
          nlo = (int64_t)s.misc[M_PLO] - a.W + 1;
          nhi = (int64_t)s.misc[M_PHI] + 1;
        }
        if (n + 2 > kStackCap || (!split_hash && nhi - nlo <= 1)) {
          win_status(a, LMS_ECAPACITY);
          s.misc[M_SSIZE] = 0;  // the call's result is void: the item stops here
        } else if (split_hash) {
          const uint64_t mid = rlo + (rhi - rlo) / 2;
          push(n, rlo, mid, elo, ehi);
          push(n + 1, mid, rhi, elo, ehi);
          s.misc[M_SSIZE] = n + 2;
        } else {
          const int64_t mid = nlo + (nhi - nlo) / 2;
          push(n, rlo, rhi, nlo, mid);
          push(n + 1, rlo, rhi, mid, nhi);
          s.misc[M_SSIZE] = n + 2;
        }
      }
      __syncthreads();
      continue;
    }
    if (a.R == 1 && a.W == 1) {
      emit_tumbling<MA>(a, s, b0);  // the inserted panes are exactly the windows to emit
    } else {
      // windows w whose first pane w * R lies in [elo, ehi)
      const int64_t wmin = any ? INT64_MIN : fdiv(elo + a.R - 1, a.R, a.inv_R);
      const int64_t wmax = any ? INT64_MAX : fdiv(ehi + a.R - 1, a.R, a.inv_R) - 1;
      emit_sliding<MA>(a, s, b0, wmin, wmax);
    }
    __syncthreads();
  }
}

// Writes the groups in the LDS tables as partial records into the partition's
// partial region [start, ...), reserving their slots with one global atomic.
template <int MA>
__device__ void flush_partials(const WinArgs& a, Lds& s, const Item& it) {
  // per-wave counts, one reservation, then barrier-free ballot-ranked writes
  // (the slot layout of emit_tumbling)
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t below = (1ull << lane) - 1;
  uint32_t mine = 0;
  for (int g0 = (int)wave * 64; g0 < a.eg; g0 += kAggTPB) {
    const int g = g0 + (int)lane;
    mine += (uint32_t)__popcll(__ballot(g < a.eg && s.gid[g] != kEmptyGid));
  }
  if (lane == 0) s.scan[wave] = mine;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < kAggTPB / 64; ++w) {
      const uint32_t v = s.scan[w];
      s.scan[w] = t;
      t += v;
    }
    s.misc[M_PC] = t ? a.pinfo[it.p].start + atomicAdd(&a.pfill[it.p], t) : 0u;
    s.scan[kAggTPB / 64] = t;
  }
  __syncthreads();
  if (s.scan[kAggTPB / 64] != 0) {
    uint32_t run = s.misc[M_PC] + s.scan[wave];
    for (int g0 = (int)wave * 64; g0 < a.eg; g0 += kAggTPB) {
      const int g = g0 + (int)lane;
      const bool occ = g < a.eg && s.gid[g] != kEmptyGid;
      const uint64_t m = __ballot(occ);
      const uint32_t e = run + (uint32_t)__popcll(m & below);
      run += (uint32_t)__popcll(m);
      if (occ) {
        const uint64_t gid = s.gid[g];
        a.pkey[e] = key_of(a, s, (uint32_t)(gid >> 32));
        a.ppane[e] = (uint32_t)gid;
        a.pcnt[e] = s.gcnt[g];
#pragma unroll
        for (int k = 0; k < MA; ++k)
          if (k < a.nacc) a.pacc[k][e] = s.acc[(size_t)k * a.eg + g];
      }
    }
  }
  __syncthreads();
}

// One piece of a split partition: aggregate its rows into partial records.
// When a table fills up, the tables are flushed and the rows that did not fit
// are inserted again into the emptied tables (at most one per thread, so they
// always fit).
template <int MA>
__device__ void aggregate_piece(const WinArgs& a, Lds& s, const Item& it) {
  if (threadIdx.x == 0) s.misc[M_OVF] = 0;
  clear_tables<MA>(a, s);
  __syncthreads();
  Elem<MA> nxt;
  if (it.lo + threadIdx.x < it.hi) load_row<MA>(a, it.lo + threadIdx.x, nxt);
  for (uint32_t b = it.lo; b < it.hi; b += kAggTPB) {
    const uint32_t e = b + threadIdx.x;
    bool pending = false;
    Elem<MA> x = nxt;
    uint64_t h = 0;
    if (e < it.hi) {  // converted before the next round's loads are issued (see aggregate_and_emit)
      finish_row<MA>(a, x);
      h = fmix64((uint64_t)x.key);
    }
    settle<MA>(x);
    if (e + kAggTPB < it.hi) load_row<MA>(a, e + kAggTPB, nxt);  // prefetch the next round
    if (e < it.hi) {
      if (!insert<MA>(a, s, x, h)) {
        pending = true;
        s.misc[M_OVF] = 1;
      }
    }
    __syncthreads();
    const bool o = s.misc[M_OVF] != 0;
    __syncthreads();
    if (o) {
      flush_partials<MA>(a, s, it);
      clear_tables<MA>(a, s);
      if (threadIdx.x == 0) s.misc[M_OVF] = 0;
      __syncthreads();
      if (pending) insert<MA>(a, s, x, h);
      __syncthreads();
    }
  }
  flush_partials<MA>(a, s, it);
}

template <int MA>
__device__ void agg_item(const WinArgs& a, uint32_t item, char* lds_raw) {
  if ((int64_t)item >= a.hdr[1]) return;
  Lds s = carve_lds(lds_raw, a.ek, a.eg, a.nacc);
  const Item it = a.items[item];
  if (it.kp > 1) {
    if (!a.emit_only) aggregate_piece<MA>(a, s, it);  // a re-emission merges the records flushed before
  } else {
    Segments sg{false, it.lo, it.hi};
    aggregate_and_emit<MA>(a, s, sg);
  }
  __syncthreads();
}

template <int MA>
__device__ void merge_part(const WinArgs& a, uint32_t p, char* lds_raw, uint64_t rlo = 0, uint64_t rhi = 1ull << 32) {
  const PartInfo pi = a.pinfo[p];
  if (pi.kp <= 1) return;
  Lds s = carve_lds(lds_raw, a.ek, a.eg, a.nacc);
  Segments sg{true, pi.start, pi.start + a.pfill[p]};
  aggregate_and_emit<MA>(a, s, sg, rlo, rhi);
  __syncthreads();
}

// A split partition is merged as kMergeParts units, each taking the keys of
// one part of the key-hash range (every unit reads all the partition's partial
// records and inserts its own): the hottest partitions' merges then run on
// several CUs instead of being the kernel's critical path.
constexpr uint32_t kMergeParts = 4;

// Claims the next unit of work from a device counter (one atomic per
// workgroup; every workgroup of the launch is resident, so claiming in order
// balances items of unequal size).
__device__ __forceinline__ uint32_t claim(int64_t* counter, uint32_t* slot) {
  if (threadIdx.x == 0) *slot = (uint32_t)atomicAdd((unsigned long long*)counter, 1ull);
  __syncthreads();
  const uint32_t v = *slot;
  __syncthreads();
  return v;
}

template <int MA>
__global__ __launch_bounds__(kAggTPB, agg_waves(MA)) void k_wa_agg(WinArgs a) {
  extern __shared__ __align__(16) char lds_raw[];
  __shared__ uint32_t slot;
  const uint32_t n = (uint32_t)a.hdr[1];
  for (uint32_t item = claim(&a.hdr[2], &slot); item < n; item = claim(&a.hdr[2], &slot))
    agg_item<MA>(a, item, lds_raw);
}

template <int MA>
__global__ __launch_bounds__(kAggTPB, agg_waves(MA)) void k_wa_merge(WinArgs a) {
  extern __shared__ __align__(16) char lds_raw[];
  __shared__ uint32_t slot;
  const uint32_t n = (uint32_t)a.hdr[4] * kMergeParts;
  for (uint32_t j = claim(&a.hdr[3], &slot); j < n; j = claim(&a.hdr[3], &slot)) {
    const uint64_t part = (1ull << 32) / kMergeParts, r = j % kMergeParts;
    merge_part<MA>(a, a.splits[j / kMergeParts], lds_raw, r * part, (r + 1) * part);
  }
}


// ---- many micro-batches in one persistent launch per stage ---------------------
//
// The per-batch arguments (one WinArgs per batch, each with its own workspace
// slice and outputs) live in device memory with prefix tables that map a
// global chunk / partition / item index to its batch.  Every stage is one
// launch of a fixed grid whose workgroups loop over the global indices, so the
// launch sequence depends only on that grid and can be captured once in a
// graph and replayed after the descriptors are rewritten for the next job.

struct MultiHdr {
  uint32_t nb;
  uint32_t nchunks;     // total scan chunks
  uint32_t nparts;      // total partitions
  uint32_t nitems;      // total aggregation item slots (per batch: its bound)
  uint32_t max_nparts;  // largest partition count of a batch
  uint32_t agg_lds;     // largest aggregation LDS plan of a batch
  uint32_t max_nacc;    // largest accumulator count of a batch
  uint32_t reserved[9];
};

// Limits a launch was configured for (LDS it was given, accumulator unroll bound).
struct MultiLim {
  uint32_t parts, agg_lds, ma, pad;
};

// A job whose descriptors exceed what the launch was configured for (a graph
// replayed after a larger job was prepared) is rejected as a whole.
__device__ __forceinline__ bool multi_fits(const MultiHdr* h, MultiLim l) {
  return h->max_nparts <= l.parts && h->agg_lds <= l.agg_lds && h->max_nacc <= l.ma;
}

struct MultiView {
  const MultiHdr* hdr;
  const uint32_t* cpre;  // nb + 1 chunk prefix
  const uint32_t* ppre;  // nb + 1 partition prefix
  const uint32_t* ipre;  // nb + 1 item-slot prefix
  uint32_t* rpre;        // nb + 1 prefix of the batches' planned items (set by k_wam_real)
  uint32_t* spre;        // nb + 1 prefix of the batches' split partitions (set by k_wam_real)
  const WinArgs* args;   // nb
};

__device__ __forceinline__ MultiView multi_view(const char* desc) {
  MultiView v;
  v.hdr = (const MultiHdr*)desc;
  const uint32_t nb = v.hdr->nb;
  size_t o = sizeof(MultiHdr);
  v.cpre = (const uint32_t*)(desc + o);
  o += align_up((size_t)(nb + 1) * 4, 16);
  v.ppre = (const uint32_t*)(desc + o);
  o += align_up((size_t)(nb + 1) * 4, 16);
  v.ipre = (const uint32_t*)(desc + o);
  o += align_up((size_t)(nb + 1) * 4, 16);
  v.rpre = (uint32_t*)(desc + o);
  o += align_up((size_t)(nb + 1) * 4, 16);
  v.spre = (uint32_t*)(desc + o);
  o += align_up((size_t)(nb + 1) * 4, 16);
  v.args = (const WinArgs*)(desc + align_up(o, 16));
  return v;
}

// Batch owning global index g: the last b with pre[b] <= g.
__device__ __forceinline__ uint32_t batch_of(const uint32_t* pre, uint32_t nb, uint32_t g) {
  uint32_t lo = 0, hi = nb - 1;
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= g) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Copies batch b's arguments into the workgroup's LDS copy when it changes.
__device__ __forceinline__ void load_args(const MultiView& v, uint32_t b, WinArgs* sa, uint32_t* cur) {
  if (*cur == b) return;
  __syncthreads();
  const uint32_t* src = (const uint32_t*)&v.args[b];
  uint32_t* dst = (uint32_t*)sa;
  for (uint32_t i = threadIdx.x; i < sizeof(WinArgs) / 4; i += blockDim.x) dst[i] = src[i];
  *cur = b;
  __syncthreads();
}

__global__ void k_wam_init(const char* desc, MultiLim lim) {
  const MultiView v = multi_view(desc);
  const bool fits = multi_fits(v.hdr, lim);
  for (uint32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < v.hdr->nb; b += gridDim.x * blockDim.x) {
    init_batch(v.args[b]);
    if (!fits) v.args[b].d_count[1] = LMS_EINVAL;
  }
}

__global__ __launch_bounds__(kScanTPB, 5) void k_wam_hist(const char* desc, MultiLim lim) {
  extern __shared__ uint32_t hist[];
  __shared__ WinArgs sa;
  const MultiView v = multi_view(desc);
  if (!multi_fits(v.hdr, lim)) return;
  uint32_t cur = ~0u;
  const uint32_t n = v.hdr->nchunks, slots = (n + kXcds - 1) / kXcds * kXcds;
  for (uint32_t g = blockIdx.x; g < slots; g += gridDim.x) {  // gridDim.x is a multiple of 8
    const uint32_t c = xcd_chunk(g, n);
    if (c >= n) continue;
    const uint32_t b = batch_of(v.cpre, v.hdr->nb, c);
    load_args(v, b, &sa, &cur);
    hist_chunk(sa, c - v.cpre[b], hist);
  }
}

__global__ __launch_bounds__(kScanTPB) void k_wam_scan1(const char* desc, MultiLim lim) {
  __shared__ uint32_t scratch[kScanTPB / 64 + 1];
  __shared__ WinArgs sa;
  const MultiView v = multi_view(desc);
  if (!multi_fits(v.hdr, lim)) return;
  uint32_t cur = ~0u;
  // a contiguous run of partitions per workgroup: the batch (and its argument
  // copy) changes only at batch boundaries
  const uint32_t n = v.hdr->nparts, per = (n + gridDim.x - 1) / gridDim.x;
  const uint32_t g0 = min(n, blockIdx.x * per), g1 = min(n, g0 + per);
  uint32_t b = g0 < g1 ? batch_of(v.ppre, v.hdr->nb, g0) : 0;
  for (uint32_t g = g0; g < g1; ++g) {
    while (g >= v.ppre[b + 1]) ++b;
    load_args(v, b, &sa, &cur);
    scan1_part(sa, (int)(g - v.ppre[b]), scratch);
    __syncthreads();
  }
}

__global__ __launch_bounds__(kPlanTPB) void k_wam_scanp(const char* desc, MultiLim lim) {
  __shared__ uint32_t r[kMaxParts], st[kMaxParts], kc[kMaxParts], base[kMaxParts];
  __shared__ uint32_t scratch[kPlanTPB / 64 + 1];
  __shared__ WinArgs sa;
  const MultiView v = multi_view(desc);
  if (!multi_fits(v.hdr, lim)) return;
  uint32_t cur = ~0u;
  for (uint32_t b = blockIdx.x; b < v.hdr->nb; b += gridDim.x) {
    load_args(v, b, &sa, &cur);
    plan_items(sa, r, st, kc, base, scratch);
  }
}

__global__ __launch_bounds__(kScanTPB) void k_wam_scan2(const char* desc, MultiLim lim) {
  __shared__ uint32_t scratch[kScanTPB / 64 + 1];
  __shared__ WinArgs sa;
  const MultiView v = multi_view(desc);
  if (!multi_fits(v.hdr, lim)) return;
  uint32_t cur = ~0u;
  const uint32_t n = v.hdr->nparts, per = (n + gridDim.x - 1) / gridDim.x;  // as in k_wam_scan1
  const uint32_t g0 = min(n, blockIdx.x * per), g1 = min(n, g0 + per);
  uint32_t b = g0 < g1 ? batch_of(v.ppre, v.hdr->nb, g0) : 0;
  for (uint32_t g = g0; g < g1; ++g) {
    while (g >= v.ppre[b + 1]) ++b;
    load_args(v, b, &sa, &cur);
    scan2_part(sa, (int)(g - v.ppre[b]), scratch);
  }
}

// Prefixes of the batches' planned items and split partitions (after the
// planner), so the aggregation and merge stages visit only real work.  One
// workgroup; each thread sums a run of consecutive batches.
__global__ __launch_bounds__(kPlanTPB) void k_wam_real(const char* desc, MultiLim lim) {
  __shared__ uint32_t si[kPlanTPB], ss[kPlanTPB];
  __shared__ uint32_t scratch[kPlanTPB / 64 + 1];
  const MultiView v = multi_view(desc);
  if (!multi_fits(v.hdr, lim)) return;
  const uint32_t nb = v.hdr->nb;
  const uint32_t per = (nb + kPlanTPB - 1) / kPlanTPB;
  const uint32_t b0 = min(nb, threadIdx.x * per), b1 = min(nb, b0 + per);
  uint32_t ci = 0, cs = 0;
  for (uint32_t b = b0; b < b1; ++b) {
    ci += (uint32_t)v.args[b].hdr[1];
    cs += (uint32_t)v.args[b].hdr[4];
  }
  si[threadIdx.x] = ci;
  ss[threadIdx.x] = cs;
  __syncthreads();
  const uint32_t ti = block_scan_array<kPlanTPB>(si, kPlanTPB, scratch);
  const uint32_t ts = block_scan_array<kPlanTPB>(ss, kPlanTPB, scratch);
  uint32_t ri = si[threadIdx.x], rs = ss[threadIdx.x];
  for (uint32_t b = b0; b < b1; ++b) {
    v.rpre[b] = ri;
    v.spre[b] = rs;
    ri += (uint32_t)v.args[b].hdr[1];
    rs += (uint32_t)v.args[b].hdr[4];
  }
  if (threadIdx.x == 0) {
    v.rpre[nb] = ti;
    v.spre[nb] = ts;
  }
}

template <int MA>
__global__ __launch_bounds__(kScatterTPB) void k_wam_scatter(const char* desc, MultiLim lim) {
  extern __shared__ uint32_t cursor[];
  __shared__ WinArgs sa;
  const MultiView v = multi_view(desc);
  if (!multi_fits(v.hdr, lim)) return;
  uint32_t cur = ~0u;
  const uint32_t n = v.hdr->nchunks, slots = (n + kXcds - 1) / kXcds * kXcds;
  for (uint32_t g = blockIdx.x; g < slots; g += gridDim.x) {
    const uint32_t c = xcd_chunk(g, n);
    if (c >= n) continue;
    const uint32_t b = batch_of(v.cpre, v.hdr->nb, c);
    load_args(v, b, &sa, &cur);
    scatter_chunk<MA>(sa, c - v.cpre[b], cursor);
  }
}

template <int MA>
__global__ __launch_bounds__(kAggTPB, agg_waves(MA)) void k_wam_agg(const char* desc, MultiLim lim) {
  extern __shared__ __align__(16) char lds_raw[];
  __shared__ WinArgs sa;
  const MultiView v = multi_view(desc);
  if (!multi_fits(v.hdr, lim)) return;
  uint32_t cur = ~0u;
  // only the items the planner made (most of each batch's item slots stay empty)
  const uint32_t nreal = v.rpre[v.hdr->nb];
  for (uint32_t g = blockIdx.x; g < nreal; g += gridDim.x) {
    const uint32_t b = batch_of(v.rpre, v.hdr->nb, g);
    load_args(v, b, &sa, &cur);
    agg_item<MA>(sa, g - v.rpre[b], lds_raw);
  }
}

template <int MA>
__global__ __launch_bounds__(kAggTPB, agg_waves(MA)) void k_wam_merge(const char* desc, MultiLim lim) {
  extern __shared__ __align__(16) char lds_raw[];
  __shared__ WinArgs sa;
  const MultiView v = multi_view(desc);
  if (!multi_fits(v.hdr, lim)) return;
  uint32_t cur = ~0u;
  // only the split partitions, in each batch's claim order
  const uint32_t nsplit = v.spre[v.hdr->nb];
  for (uint32_t g = blockIdx.x; g < nsplit; g += gridDim.x) {
    const uint32_t b = batch_of(v.spre, v.hdr->nb, g);
    load_args(v, b, &sa, &cur);
    merge_part<MA>(sa, sa.splits[g - v.spre[b]], lds_raw);
  }
}

// ---- re-emission from an intact workspace --------------------------------------
//
// The staged records, the item plan and the split partitions' partial records
// stay in the workspace after a call, so its groups can be emitted again into
// other outputs without reading the input columns: the aggregation items are
// re-run (pieces excepted: their partial records are already flushed) and the
// split partitions merged again.

struct EmitOut {
  int64_t* okey;
  int64_t* ows;
  void* oagg[kMaxAggs];
  int64_t cap;
  int64_t* d_count;
  int32_t nagg;
  int32_t reserved;
};

__global__ void k_wa_emit_init(char* ws, EmitOut o) {
  if (threadIdx.x != 0) return;
  int64_t* const hdr = (int64_t*)ws;
  WinArgs* const sv = (WinArgs*)(ws + kSavedOff);
  o.d_count[0] = 0;
  const bool ok = hdr[6] == kSavedMagic && sv->hdr == hdr && sv->nagg == o.nagg;
  hdr[7] = ok ? 1 : 0;
  if (!ok) {
    o.d_count[1] = LMS_EINVAL;
    return;
  }
  o.d_count[1] = hdr[5];  // the status the call's own kernels set
  WinArgs* const ea = sv + 1;
  *ea = *sv;
  ea->okey = o.okey;
  ea->ows = o.ows;
  for (int k = 0; k < kMaxAggs; ++k) ea->oagg[k] = o.oagg[k];
  ea->cap = o.cap;
  ea->d_count = o.d_count;
  ea->emit_only = 1;
  hdr[2] = 0;
  hdr[3] = 0;
}

// The re-emission's arguments, copied into the workgroup's LDS.
__device__ __forceinline__ bool load_emit_args(const char* ws, WinArgs* sa) {
  if (((const int64_t*)ws)[7] != 1) return false;
  const uint32_t* src = (const uint32_t*)((const WinArgs*)(ws + kSavedOff) + 1);
  uint32_t* dst = (uint32_t*)sa;
  for (uint32_t i = threadIdx.x; i < sizeof(WinArgs) / 4; i += blockDim.x) dst[i] = src[i];
  __syncthreads();
  return true;
}

template <int MA>
__global__ __launch_bounds__(kAggTPB, agg_waves(MA)) void k_wa_agg_again(const char* ws) {
  extern __shared__ __align__(16) char lds_raw[];
  __shared__ WinArgs sa;
  __shared__ uint32_t slot;
  if (!load_emit_args(ws, &sa)) return;
  const uint32_t n = (uint32_t)sa.hdr[1];
  for (uint32_t item = claim(&sa.hdr[2], &slot); item < n; item = claim(&sa.hdr[2], &slot))
    agg_item<MA>(sa, item, lds_raw);
}

template <int MA>
__global__ __launch_bounds__(kAggTPB, agg_waves(MA)) void k_wa_merge_again(const char* ws) {
  extern __shared__ __align__(16) char lds_raw[];
  __shared__ WinArgs sa;
  __shared__ uint32_t slot;
  if (!load_emit_args(ws, &sa)) return;
  const uint32_t n = (uint32_t)sa.hdr[4] * kMergeParts;
  for (uint32_t j = claim(&sa.hdr[3], &slot); j < n; j = claim(&sa.hdr[3], &slot)) {
    const uint64_t part = (1ull << 32) / kMergeParts, r = j % kMergeParts;
    merge_part<MA>(sa, sa.splits[j / kMergeParts], lds_raw, r * part, (r + 1) * part);
  }
}

// ---- host planning -------------------------------------------------------------

int64_t next_pow2(int64_t x) {
  int64_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

int ilog2(int64_t x) {
  int b = 0;
  while ((int64_t(1) << b) < x) ++b;
  return b;
}

struct Plan {
  int64_t n;
  int64_t chunk;
  int g1;
  int nparts, pbits;
  int64_t rs;
  int max_items;
  int ek, eg;
  size_t lds;
  int nval, nacc;
};

int64_t gcd64(int64_t x, int64_t y) {
  while (y) {
    int64_t t = x % y;
    x = y;
    y = t;
  }
  return x;
}

lms_tuning g_tuning{0, 0, 0, 0, 0, 0};

// Workgroup slots of a launch over n chunks (a multiple of the 8 XCDs).
unsigned xcd_slots(int n) { return (unsigned)((n + kXcds - 1) / kXcds * kXcds); }

// Bytes of a staged record for nval value columns, whatever their widths.
size_t rec_bound(int nval) { return align_up(8 + 4 + 8 * (size_t)nval, 8); }

// Unroll bound of the per-accumulator loops (the kernels are instantiated for 2, 4, 6, 8).
int acc_bound(int nacc) { return nacc <= 2 ? 2 : nacc <= 4 ? 4 : nacc <= 6 ? 6 : 8; }

Plan make_plan(int64_t n, int nval, int nacc) {
  Plan p{};
  p.n = n;
  if (g_tuning.chunk_rows > 0) p.chunk = std::min<int64_t>(kMaxChunk, next_pow2(g_tuning.chunk_rows));
  else p.chunk = std::min<int64_t>(kMaxChunk, std::max<int64_t>(2048, next_pow2((n + 1023) / 1024)));
  p.g1 = (int)((n + p.chunk - 1) / p.chunk);
  // the LDS group table sets the scale: by default a partition targets 8 rows
  // per table slot and an aggregation piece 4 (16384 and 8192 at 2048 slots);
  // a batch too small to fill kMinParts partitions that way targets fewer rows
  // per partition (down to 2048), so its items run on that many CUs at once
  // instead of on a few: a micro-batch's latency is its longest item's
  p.eg = g_tuning.lds_groups > 0 ? g_tuning.lds_groups : 2048;
  p.ek = p.eg / 2;
  const int64_t part_rows = g_tuning.part_rows > 0
                                ? g_tuning.part_rows
                                : std::min<int64_t>(8 * (int64_t)p.eg,
                                                    std::max<int64_t>(2048, (n + kMinParts - 1) / kMinParts));
  p.nparts = (int)std::min<int64_t>(kMaxParts, std::max<int64_t>(8, next_pow2((n + part_rows - 1) / part_rows)));
  p.pbits = ilog2(p.nparts);
  p.rs = g_tuning.piece_rows > 0 ? g_tuning.piece_rows : 4 * (int64_t)p.eg;
  p.max_items = p.nparts + (int)((n + p.rs - 1) / p.rs);
  while (lds_bytes(p.ek, p.eg, nacc) + kArgsLds > (size_t)kLdsLimit && p.eg > 1024) {
    p.eg /= 2;
    p.ek /= 2;
  }
  p.lds = lds_bytes(p.ek, p.eg, nacc);
  p.nval = nval;
  p.nacc = nacc;
  return p;
}

// Carves the workspace; with base == nullptr only computes the size.
size_t carve_workspace(const Plan& p, void* base, WinArgs* a) {
  WsCarver c(base);
  int64_t* hdr = c.take<int64_t>(8);
  WinArgs* saved = c.take<WinArgs>(2);  // at kSavedOff
  uint32_t* splits = c.take<uint32_t>(p.nparts);
  uint32_t* H = c.take<uint32_t>((size_t)p.nparts * p.g1);
  uint32_t* Off = c.take<uint32_t>((size_t)p.nparts * p.g1);
  uint32_t* Rp = c.take<uint32_t>(p.nparts);
  PartInfo* pinfo = c.take<PartInfo>(p.nparts);
  Item* items = c.take<Item>(p.max_items);
  uint32_t* pfill = c.take<uint32_t>(p.nparts);
  uint64_t* pmask = c.take<uint64_t>((size_t)(p.n + 63) / 64 + 1);
  char* srec = c.take<char>((size_t)p.n * rec_bound(p.nval) + 8);  // + one spare word
  int64_t* pkey = c.take<int64_t>(p.n);
  uint32_t* ppane = c.take<uint32_t>(p.n);
  uint32_t* pcnt = c.take<uint32_t>(p.n);
  uint64_t* pacc[kMaxAggs] = {};
  for (int k = 0; k < p.nacc; ++k) pacc[k] = c.take<uint64_t>(p.n);
  if (a) {
    a->hdr = hdr;
    a->saved = saved;
    a->splits = splits;
    a->H = H;
    a->Off = Off;
    a->Rp = Rp;
    a->pinfo = pinfo;
    a->items = items;
    a->pfill = pfill;
    a->pmask = pmask;
    a->srec = srec;
    a->pkey = pkey;
    a->ppane = ppane;
    a->pcnt = pcnt;
    for (int k = 0; k < kMaxAggs; ++k) a->pacc[k] = pacc[k];
  }
  return c.size();
}

// Resolves the aggregate list into staged value columns and accumulators.
int resolve_aggs(const lms_batch* in, const lms_proj* projs, int32_t nproj, const lms_agg* aggs, int32_t nagg,
                 WinArgs* a) {
  if (nagg < 0 || nagg > kMaxAggs) return set_error(LMS_EINVAL, "nagg %d outside [0, %d]", nagg, kMaxAggs);
  if (nagg > 0 && !aggs) return set_error(LMS_EINVAL, "aggs is NULL");
  const int next = in->ncols + (projs ? nproj : 0);
  a->nagg = nagg;
  a->nval = 0;
  a->nacc = 0;
  for (int k = 0; k < nagg; ++k) {
    const int fn = aggs[k].fn;
    if (fn < LMS_COUNT || fn > LMS_AVG) return set_error(LMS_EINVAL, "aggregate %d has bad function %d", k, fn);
    a->afn[k] = fn;
    a->aacc[k] = -1;
    if (fn == LMS_COUNT) continue;
    const int c = aggs[k].col;
    if (c < 0 || c >= next) return set_error(LMS_EINVAL, "aggregate %d column %d out of range", k, c);
    const int dt = c < in->ncols ? in->cols[c].dtype : in->cols[projs[c - in->ncols].src].dtype;
    if (fn != LMS_AVG && !(dt == LMS_I32 || dt == LMS_I64))
      return set_error(LMS_EINVAL, "aggregate %d: SUM/MIN/MAX need an integer column", k);
    int v = -1;
    for (int j = 0; j < a->nval; ++j)
      if (a->vcol[j] == c) v = j;
    if (v < 0) {
      v = a->nval++;
      a->vcol[v] = c;
      a->vdt[v] = dt;
    }
    const int s = a->nacc++;
    a->accfn[s] = fn;
    a->accval[s] = v;
    a->aacc[k] = s;
  }
  // staged record: key, 8-byte values, pane, 4-byte values, padded to 8 bytes
  int off = 8;
  for (int v = 0; v < a->nval; ++v)
    if (a->vdt[v] == LMS_I64 || a->vdt[v] == LMS_F64) {
      a->voff[v] = off;
      off += 8;
    }
  a->pane_off = off;
  off += 4;
  for (int v = 0; v < a->nval; ++v)
    if (a->vdt[v] == LMS_I32 || a->vdt[v] == LMS_F32) {
      a->voff[v] = off;
      off += 4;
    }
  a->rec = (int32_t)align_up((size_t)off, 8);
  return LMS_OK;
}

int validate_window(const lms_batch* in, int32_t key_col, const lms_window* w) {
  if (!in) return set_error(LMS_EINVAL, "input batch is NULL");
  if (!w) return set_error(LMS_EINVAL, "window is NULL");
  if (key_col < 0 || key_col >= in->ncols) return set_error(LMS_EINVAL, "key column %d out of range", key_col);
  if (!in->cols) return set_error(LMS_EINVAL, "cols is NULL");
  const int kdt = in->cols[key_col].dtype;
  if (kdt != LMS_I32 && kdt != LMS_I64) return set_error(LMS_EINVAL, "key column must be integer");
  if (w->ts_col < 0 || w->ts_col >= in->ncols) return set_error(LMS_EINVAL, "ts column %d out of range", w->ts_col);
  const int tdt = in->cols[w->ts_col].dtype;
  if (tdt != LMS_I32 && tdt != LMS_I64) return set_error(LMS_EINVAL, "ts column must be integer");
  if (w->len <= 0 || w->len >= (int64_t(1) << 31)) return set_error(LMS_EINVAL, "window length must be in (0, 2^31)");
  if (w->slide < 0 || w->slide > w->len) return set_error(LMS_EINVAL, "slide must be in [0, len]");
  if (in->nrows >= (int64_t(1) << 31)) return set_error(LMS_EINVAL, "micro-batch must have < 2^31 rows");
  return LMS_OK;
}

int num_cus() {
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

template <int MA>
void launch_tail(const Plan& p, const WinArgs& a, size_t plds, hipStream_t st) {
  static const int attr_rc = [] {
    int rc = check_hip(hipFuncSetAttribute((const void*)k_wa_agg<MA>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           kLdsLimit - kArgsLds), "LDS attribute");
    if (!rc)
      rc = check_hip(hipFuncSetAttribute((const void*)k_wa_merge<MA>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         kLdsLimit - kArgsLds), "LDS attribute");
    return rc;
  }();
  if (attr_rc) return;  // the launch error is reported by the caller's hipGetLastError
  // the aggregation kernels claim work from counters, so they run as many
  // workgroups as the CUs hold at once: one per CU (a 1024-thread workgroup
  // already fills each SIMD's register budget at 4 waves)
  const int resident = num_cus();
  if constexpr (MA <= 6) {
    static const int st_rc = check_hip(hipFuncSetAttribute((const void*)k_wa_scatter_st<MA>,
                                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)kStLds),
                                       "LDS attribute");
    if (st_rc) return;
    LMS_LAUNCH("k_wa_scatter", k_wa_scatter_st<MA>, dim3(xcd_slots(p.g1)), dim3(kStTPB), kStLds, st, a);
  } else {
    LMS_LAUNCH("k_wa_scatter", k_wa_scatter<MA>, dim3(xcd_slots(p.g1)), dim3(kScatterTPB),
               hist_lds(p.nparts, p.chunk), st, a);
  }
  LMS_LAUNCH("k_wa_agg", k_wa_agg<MA>, dim3(std::min(p.max_items, resident)), dim3(kAggTPB), p.lds, st, a);
  LMS_LAUNCH("k_wa_merge", k_wa_merge<MA>, dim3(std::min(p.nparts, resident)), dim3(kAggTPB), p.lds, st, a);
}

}  // namespace
}  // namespace lms

using namespace lms;

extern "C" int64_t lms_window_agg_pane_limit(int32_t nagg) {
  int nacc = std::max(0, std::min<int>(nagg, kMaxAggs));
  return make_plan(1, 1, nacc).eg;
}

extern "C" size_t lms_window_agg_workspace(const lms_batch* in, int32_t key_col, const lms_window* w,
                                           const lms_agg* aggs, int32_t nagg) {
  if (validate_window(in, key_col, w) != LMS_OK) return 0;
  WinArgs a{};
  // projections are not known here: every value column is sized at 8 bytes.
  int nval = 0, nacc = 0;
  if (nagg > 0 && aggs) {
    int cols[kMaxAggs];
    for (int k = 0; k < nagg && k < kMaxAggs; ++k) {
      if (aggs[k].fn == LMS_COUNT) continue;
      ++nacc;
      bool seen = false;
      for (int j = 0; j < nval; ++j) seen |= cols[j] == aggs[k].col;
      if (!seen) cols[nval++] = aggs[k].col;
    }
  }
  (void)a;
  return carve_workspace(make_plan(in->nrows, nval, nacc), nullptr, nullptr);
}

namespace lms {
namespace {

// Validates one batch's call and fills its kernel arguments, carving `workspace`.
int setup_args(const lms_batch* in, const lms_pred* preds, int32_t npred, const lms_proj* projs, int32_t nproj,
               int32_t key_col, const lms_window* w, const lms_agg* aggs, int32_t nagg, const lms_groups* out,
               int64_t* d_count, void* workspace, size_t ws_bytes, WinArgs* pa, Plan* pplan) {
  int rc = validate_window(in, key_col, w);
  if (rc) return rc;
  WinArgs& a = *pa;
  a = WinArgs{};
  rc = build_query(in, preds, npred, projs, nproj, &a.q);
  if (rc) return rc;
  rc = resolve_aggs(in, projs, nproj, aggs, nagg, &a);
  if (rc) return rc;
  if (!out) return set_error(LMS_EINVAL, "output groups is NULL");
  if (out->cap < 0) return set_error(LMS_EINVAL, "negative output capacity");
  if (out->cap > 0 && (!out->key || !out->wstart)) return set_error(LMS_EINVAL, "output key/wstart is NULL");
  if (nagg > 0 && !out->aggs) return set_error(LMS_EINVAL, "output aggs is NULL");
  for (int k = 0; k < nagg; ++k)
    if (out->cap > 0 && !out->aggs[k]) return set_error(LMS_EINVAL, "output aggregate %d is NULL", k);
  if (!d_count) return set_error(LMS_EINVAL, "d_count is NULL");
  const Plan p = make_plan(in->nrows, a.nval, a.nacc);
  const size_t need = carve_workspace(p, nullptr, nullptr);
  if (!workspace || ws_bytes < need)
    return set_error(LMS_ENOMEM, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
  carve_workspace(p, workspace, &a);
  a.key_col = key_col;
  a.ts_col = w->ts_col;
  a.quads = preds_aligned(a.q) && ((uintptr_t)a.q.col[key_col] & 15) == 0 ? 1 : 0;
  a.len = w->len;
  a.slide = w->slide == 0 ? w->len : w->slide;
  a.origin = w->origin;
  a.pane = gcd64(a.len, a.slide);
  a.R = a.slide / a.pane;
  a.W = a.len / a.pane;
  a.inv_pane = 1.0 / (double)a.pane;
  a.inv_R = 1.0 / (double)a.R;
  a.pbits = p.pbits;
  a.nparts = p.nparts;
  a.g1 = p.g1;
  a.max_items = p.max_items;
  a.ek = p.ek;
  a.eg = p.eg;
  a.chunk = p.chunk;
  a.rs = p.rs;
  a.okey = out->key;
  a.ows = out->wstart;
  for (int k = 0; k < nagg; ++k) a.oagg[k] = out->aggs[k];
  a.cap = out->cap;
  a.d_count = d_count;
  *pplan = p;
  return LMS_OK;
}


// Pinned staging of the multi-batch descriptors: the upload is asynchronous,
// so the next prepare waits for the previous upload before reusing the buffer.
struct DescStage {
  std::mutex mu;
  char* host = nullptr;
  size_t cap = 0;
  hipEvent_t done = nullptr;
  bool pending = false;
};
DescStage g_stage;

size_t multi_desc_bytes(int nb) {
  size_t o = sizeof(MultiHdr) + 5 * align_up((size_t)(nb + 1) * 4, 16);
  return align_up(align_up(o, 16) + (size_t)nb * sizeof(WinArgs), 256);
}

template <int MA>
int launch_multi(const lms_multi_config& c, const char* desc, hipStream_t st) {
  static const int attr_rc = [] {
    int rc = check_hip(hipFuncSetAttribute((const void*)k_wam_agg<MA>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           kLdsLimit - kArgsLds), "LDS attribute");
    if (!rc)
      rc = check_hip(hipFuncSetAttribute((const void*)k_wam_merge<MA>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                         kLdsLimit - kArgsLds), "LDS attribute");
    return rc;
  }();
  if (attr_rc) return attr_rc;
  const size_t plds = (size_t)c.max_nparts * 4;
  const MultiLim lim{(uint32_t)c.max_nparts, (uint32_t)c.agg_lds, (uint32_t)MA, 0};
  LMS_LAUNCH("k_wam_init", k_wam_init, dim3(4), dim3(256), 0, st, desc, lim);
  LMS_LAUNCH("k_wam_hist", k_wam_hist, dim3(c.grid_scan), dim3(kScanTPB), hist_lds(c.max_nparts, kMaxChunk), st,
             desc, lim);
  LMS_LAUNCH("k_wam_scan1", k_wam_scan1, dim3(c.grid_scan), dim3(kScanTPB), 0, st, desc, lim);
  LMS_LAUNCH("k_wam_scanp", k_wam_scanp, dim3(c.grid_scan), dim3(kPlanTPB), 0, st, desc, lim);
  LMS_LAUNCH("k_wam_real", k_wam_real, dim3(1), dim3(kPlanTPB), 0, st, desc, lim);
  LMS_LAUNCH("k_wam_scan2", k_wam_scan2, dim3(c.grid_scan), dim3(kScanTPB), 0, st, desc, lim);
  LMS_LAUNCH("k_wam_scatter", k_wam_scatter<MA>, dim3(c.grid_scan), dim3(kScatterTPB), hist_lds(c.max_nparts, kMaxChunk),
             st, desc, lim);
  LMS_LAUNCH("k_wam_agg", k_wam_agg<MA>, dim3(c.grid_agg), dim3(kAggTPB), (size_t)c.agg_lds, st, desc, lim);
  LMS_LAUNCH("k_wam_merge", k_wam_merge<MA>, dim3(c.grid_agg), dim3(kAggTPB), (size_t)c.agg_lds, st, desc, lim);
  return LMS_OK;
}

}  // namespace
}  // namespace lms

extern "C" int lms_window_agg(const lms_batch* in, const lms_pred* preds, int32_t npred, const lms_proj* projs,
                              int32_t nproj, int32_t key_col, const lms_window* w, const lms_agg* aggs, int32_t nagg,
                              const lms_groups* out, int64_t* d_count, void* workspace, size_t ws_bytes,
                              lms_stream stream) {
  WinArgs a;
  Plan p;
  int rc = setup_args(in, preds, npred, projs, nproj, key_col, w, aggs, nagg, out, d_count, workspace, ws_bytes, &a, &p);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  if (in->nrows == 0) LMS_LAUNCH("k_wa_init", k_wa_init, dim3(1), dim3(64), 0, st, a);
  if (in->nrows > 0) {
    const size_t plds = (size_t)p.nparts * 4;
    LMS_LAUNCH("k_wa_hist", k_wa_hist, dim3(xcd_slots(p.g1)), dim3(kScanTPB), hist_lds(p.nparts, p.chunk), st, a);
    if (p.g1 <= kSmallChunks) {
      LMS_LAUNCH("k_wa_scans", k_wa_scans, dim3(1), dim3(kPlanTPB), 0, st, a);
    } else {
      LMS_LAUNCH("k_wa_scan1", k_wa_scan1, dim3(p.nparts), dim3(kScanTPB), 0, st, a);
      LMS_LAUNCH("k_wa_scanp", k_wa_scanp, dim3(1), dim3(kPlanTPB), 0, st, a);
      LMS_LAUNCH("k_wa_scan2", k_wa_scan2, dim3(p.nparts), dim3(kScanTPB), 0, st, a);
    }
    // loops over accumulators are unrolled to the smallest bound covering them
    const int ma = acc_bound(a.nacc);
    if (ma == 2) launch_tail<2>(p, a, plds, st);
    else if (ma == 4) launch_tail<4>(p, a, plds, st);
    else if (ma == 6) launch_tail<6>(p, a, plds, st);
    else launch_tail<8>(p, a, plds, st);
  }
  return check_hip(hipGetLastError(), "window_agg launch");
}

extern "C" int lms_window_agg_emit(const lms_groups* out, int32_t nagg, int64_t* d_count, void* workspace,
                                   size_t ws_bytes, lms_stream stream) {
  if (!out) return set_error(LMS_EINVAL, "output groups is NULL");
  if (out->cap < 0) return set_error(LMS_EINVAL, "negative output capacity");
  if (out->cap > 0 && (!out->key || !out->wstart)) return set_error(LMS_EINVAL, "output key/wstart is NULL");
  if (nagg < 0 || nagg > kMaxAggs) return set_error(LMS_EINVAL, "nagg %d outside [0, %d]", nagg, kMaxAggs);
  if (nagg > 0 && !out->aggs) return set_error(LMS_EINVAL, "output aggs is NULL");
  for (int k = 0; k < nagg; ++k)
    if (out->cap > 0 && !out->aggs[k]) return set_error(LMS_EINVAL, "output aggregate %d is NULL", k);
  if (!d_count) return set_error(LMS_EINVAL, "d_count is NULL");
  if (!workspace || ws_bytes < kSavedOff + 2 * sizeof(WinArgs))
    return set_error(LMS_EINVAL, "workspace is not one a lms_window_agg call filled");
  static const int attr_rc = [] {
    int rc = check_hip(hipFuncSetAttribute((const void*)k_wa_agg_again<kMaxAggs>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, kLdsLimit - kArgsLds),
                       "LDS attribute");
    if (!rc)
      rc = check_hip(hipFuncSetAttribute((const void*)k_wa_merge_again<kMaxAggs>,
                                         hipFuncAttributeMaxDynamicSharedMemorySize, kLdsLimit - kArgsLds),
                     "LDS attribute");
    return rc;
  }();
  if (attr_rc) return attr_rc;
  EmitOut o{};
  o.okey = out->key;
  o.ows = out->wstart;
  for (int k = 0; k < nagg; ++k) o.oagg[k] = out->aggs[k];
  o.cap = out->cap;
  o.d_count = d_count;
  o.nagg = nagg;
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)workspace;
  // the kernels take the accumulator count from the saved arguments, so the
  // widest unroll serves every call
  const int resident = num_cus();
  LMS_LAUNCH("k_wa_emit_init", k_wa_emit_init, dim3(1), dim3(64), 0, st, ws, o);
  LMS_LAUNCH("k_wa_agg_again", k_wa_agg_again<kMaxAggs>, dim3(resident), dim3(kAggTPB), kLdsLimit - kArgsLds, st,
             (const char*)ws);
  LMS_LAUNCH("k_wa_merge_again", k_wa_merge_again<kMaxAggs>, dim3(resident), dim3(kAggTPB), kLdsLimit - kArgsLds,
             st, (const char*)ws);
  return check_hip(hipGetLastError(), "window_agg_emit launch");
}

extern "C" int lms_set_tuning(const lms_tuning* t) {
  if (!t) {
    g_tuning = lms_tuning{0, 0, 0, 0, 0, 0};
    return LMS_OK;
  }
  if (t->chunk_rows < 0 || t->part_rows < 0 || t->piece_rows < 0 || t->grid_per_cu < 0 || t->lds_groups < 0)
    return set_error(LMS_EINVAL, "tuning values must be >= 0");
  if (t->piece_rows > 0 && t->piece_rows < 1024) return set_error(LMS_EINVAL, "piece_rows must be >= 1024");
  if (t->lds_groups != 0 && (t->lds_groups < 1024 || t->lds_groups > 2048 || (t->lds_groups & (t->lds_groups - 1))))
    return set_error(LMS_EINVAL, "lds_groups must be 0, 1024 or 2048");
  g_tuning = *t;
  return LMS_OK;
}

extern "C" int lms_get_tuning(lms_tuning* t) {
  if (!t) return set_error(LMS_EINVAL, "NULL");
  *t = g_tuning;
  return LMS_OK;
}

extern "C" size_t lms_window_agg_multi_workspace(const lms_batch* batches, int32_t nbatch, int32_t key_col,
                                                 const lms_window* w, const lms_agg* aggs, int32_t nagg) {
  if (!batches || nbatch <= 0) return 0;
  size_t total = multi_desc_bytes(nbatch);
  for (int b = 0; b < nbatch; ++b) {
    const size_t one = lms_window_agg_workspace(&batches[b], key_col, w, aggs, nagg);
    if (one == 0) return 0;
    total += align_up(one, 256);
  }
  return total;
}

extern "C" int lms_window_agg_multi_prepare(const lms_batch* batches, int32_t nbatch, const lms_pred* preds,
                                            int32_t npred, const lms_proj* projs, int32_t nproj, int32_t key_col,
                                            const lms_window* w, const lms_agg* aggs, int32_t nagg,
                                            const lms_groups* outs, int64_t* d_counts, void* workspace,
                                            size_t ws_bytes, lms_multi_config* cfg, lms_stream stream) {
  if (!batches || nbatch <= 0 || !outs || !d_counts || !cfg || !workspace)
    return set_error(LMS_EINVAL, "bad multi-batch arguments");
  const size_t dbytes = multi_desc_bytes(nbatch);
  if (ws_bytes < dbytes) return set_error(LMS_ENOMEM, "workspace too small");
  std::lock_guard<std::mutex> lk(g_stage.mu);
  if (g_stage.pending) {
    int rc = check_hip(hipEventSynchronize(g_stage.done), "descriptor staging wait");
    if (rc) return rc;
    g_stage.pending = false;
  }
  if (!g_stage.done) {
    int rc = check_hip(hipEventCreateWithFlags(&g_stage.done, hipEventDisableTiming), "event create");
    if (rc) return rc;
  }
  if (g_stage.cap < dbytes) {
    if (g_stage.host) (void)hipHostFree(g_stage.host);
    g_stage.host = nullptr;
    g_stage.cap = 0;
    int rc = check_hip(hipHostMalloc((void**)&g_stage.host, dbytes, hipHostMallocDefault), "pinned staging");
    if (rc) return rc;
    g_stage.cap = dbytes;
  }
  std::memset(g_stage.host, 0, dbytes);
  char* const hbuf = g_stage.host;
  MultiHdr* hdr = (MultiHdr*)hbuf;
  hdr->nb = (uint32_t)nbatch;
  size_t o = sizeof(MultiHdr);
  uint32_t* cpre = (uint32_t*)(hbuf + o);
  o += align_up((size_t)(nbatch + 1) * 4, 16);
  uint32_t* ppre = (uint32_t*)(hbuf + o);
  o += align_up((size_t)(nbatch + 1) * 4, 16);
  uint32_t* ipre = (uint32_t*)(hbuf + o);
  o += align_up((size_t)(nbatch + 1) * 4, 16);
  o += 2 * align_up((size_t)(nbatch + 1) * 4, 16);  // item and split prefixes, set on the device
  WinArgs* args = (WinArgs*)(hbuf + align_up(o, 16));
  size_t off = dbytes;
  int max_nparts = 1, max_nacc = 0;
  uint64_t c = 0, pp = 0, it = 0;
  size_t agg_lds = 0;
  for (int b = 0; b < nbatch; ++b) {
    Plan p;
    const size_t remain = ws_bytes > off ? ws_bytes - off : 0;
    int rc = setup_args(&batches[b], preds, npred, projs, nproj, key_col, w, aggs, nagg, &outs[b], d_counts + 2 * b,
                        (char*)workspace + off, remain, &args[b], &p);
    if (rc) return rc;
    off += align_up(carve_workspace(p, nullptr, nullptr), 256);
    cpre[b] = (uint32_t)c;
    ppre[b] = (uint32_t)pp;
    ipre[b] = (uint32_t)it;
    c += (uint64_t)p.g1;
    pp += (uint64_t)p.nparts;
    it += (uint64_t)p.max_items;
    max_nparts = std::max(max_nparts, p.nparts);
    max_nacc = std::max(max_nacc, args[b].nacc);
    agg_lds = std::max(agg_lds, p.lds);
  }
  if (c >= (1ull << 32) || pp >= (1ull << 32) || it >= (1ull << 32)) return set_error(LMS_EINVAL, "job too large");
  cpre[nbatch] = (uint32_t)c;
  ppre[nbatch] = (uint32_t)pp;
  ipre[nbatch] = (uint32_t)it;
  hdr->nchunks = (uint32_t)c;
  hdr->nparts = (uint32_t)pp;
  hdr->nitems = (uint32_t)it;
  hdr->max_nparts = (uint32_t)max_nparts;
  hdr->agg_lds = (uint32_t)agg_lds;
  hdr->max_nacc = (uint32_t)max_nacc;
  cfg->nbatch = nbatch;
  cfg->ma = acc_bound(max_nacc);
  cfg->max_nparts = max_nparts;
  const int per_cu = g_tuning.grid_per_cu > 0 ? g_tuning.grid_per_cu : 4;
  cfg->grid_scan = num_cus() * per_cu;
  cfg->grid_agg = num_cus();
  cfg->reserved = 0;
  cfg->agg_lds = agg_lds;
  int rc = check_hip(hipMemcpyAsync(workspace, hbuf, dbytes, hipMemcpyHostToDevice, (hipStream_t)stream),
                     "descriptor upload");
  if (rc) return rc;
  rc = check_hip(hipEventRecord(g_stage.done, (hipStream_t)stream), "descriptor upload event");
  if (rc) return rc;
  g_stage.pending = true;
  return LMS_OK;
}

extern "C" int lms_window_agg_multi_launch(const lms_multi_config* cfg, void* workspace, lms_stream stream) {
  if (!cfg || !workspace || cfg->nbatch <= 0) return set_error(LMS_EINVAL, "bad multi-batch launch arguments");
  if (cfg->grid_scan <= 0 || cfg->grid_agg <= 0 || cfg->max_nparts <= 0 || cfg->max_nparts > kMaxParts ||
      cfg->agg_lds > (uint64_t)(kLdsLimit - kArgsLds) ||
      !(cfg->ma == 2 || cfg->ma == 4 || cfg->ma == 6 || cfg->ma == 8))
    return set_error(LMS_EINVAL, "bad multi-batch configuration");
  hipStream_t st = (hipStream_t)stream;
  const char* desc = (const char*)workspace;
  int rc = LMS_OK;
  switch (cfg->ma) {
    case 2: rc = launch_multi<2>(*cfg, desc, st); break;
    case 4: rc = launch_multi<4>(*cfg, desc, st); break;
    case 6: rc = launch_multi<6>(*cfg, desc, st); break;
    case 8: rc = launch_multi<8>(*cfg, desc, st); break;
  }
  if (rc) return rc;
  return check_hip(hipGetLastError(), "multi-batch launch");
}
