// Stream-static hash join (Table II "Join (Hash)"; the stream join of LR1,
// Table III): inner equi-join of a micro-batch against a static table.
//
// Build: open addressing with linear probing in a power-of-two table of
// 16-byte slots (key, payload, used) at load factor <= 0.5; a slot is claimed
// with one 32-bit CAS, duplicate keys take separate slots.  All slots of a key
// lie in the run of used slots that starts at its home slot, so a probe walks
// from the home slot to the first unused slot.
// Probe: one pass walks the chains (a row's walk stops at its match when the
// build found no repeated key; each lane walks its rows one after another,
// independently of the other lanes) and records per row what the write pass
// needs (a payload and a hit bit when no key repeats, else the match count
// and first payload), with per-tile totals (a tile is one wave's contiguous
// range); a scan of the tile counts; then a write pass that ranks the pairs
// of each 64-row group (by the hit mask, or a wave scan of the counts) with a
// running offset, so the pairs come out grouped by ascending probe row
// without global atomics or workgroup barriers, and touches the table again
// only for rows with several matches.
#include <algorithm>

#include "lms_internal.h"

struct JSlot {
  int64_t key;
  int32_t pay;
  uint32_t used;
};
static_assert(sizeof(JSlot) == 16, "a slot is read as one 16-byte load");

struct lms_join_table {
  JSlot* slots;
  uint64_t mask;
  int64_t nbuild;
  int64_t* d_mult;
  hipEvent_t built;
  int64_t mult_cache;
};

namespace lms {
namespace {

constexpr int kTPB = 256;
constexpr int kScanThreads = 1024;
constexpr int kProbe = 2;  // rows per lane per round of the write pass when keys repeat

__global__ void k_jb_clear(JSlot* slots, uint64_t nslots, int64_t* d_mult) {
  const uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
  if (i < nslots) {
    slots[i].key = 0;
    slots[i].pay = 0;
    slots[i].used = 0;
  }
  if (i == 0) *d_mult = 0;
}

__global__ void k_jb_insert(JSlot* slots, uint64_t mask, const void* keys, int kdt, const int32_t* pay, int64_t n) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int64_t k = load_i64(keys, kdt, j);
  uint64_t s = fmix64((uint64_t)k) & mask;
  for (uint64_t t = 0; t <= mask; ++t) {
    if (atomicCAS(&slots[s].used, 0u, 1u) == 0u) {
      slots[s].key = k;
      slots[s].pay = pay[j];
      return;
    }
    s = (s + 1) & mask;
  }
}

// Largest number of slots sharing one key.
__global__ __launch_bounds__(kTPB) void k_jb_mult(const JSlot* slots, uint64_t mask, int64_t* d_mult) {
  __shared__ uint32_t scratch[kTPB / 64 + 1];
  __shared__ uint32_t bmax;
  if (threadIdx.x == 0) bmax = 0;
  __syncthreads();
  const uint64_t i = blockIdx.x * (uint64_t)kTPB + threadIdx.x;
  uint32_t m = 0;
  if (i <= mask && slots[i].used) {
    const int64_t k = slots[i].key;
    uint64_t s = fmix64((uint64_t)k) & mask;
    for (uint64_t t = 0; t <= mask && slots[s].used; ++t) {
      m += slots[s].key == k;
      s = (s + 1) & mask;
    }
  }
  atomicMax(&bmax, m);
  __syncthreads();
  if (threadIdx.x == 0 && bmax > 0) atomicMax((unsigned long long*)d_mult, (unsigned long long)bmax);
  (void)scratch;
}

struct ProbeArgs {
  const JSlot* slots;
  uint64_t mask;
  const void* pkey;
  int32_t kdt;
  int64_t n;
  int64_t chunk;
  int32_t ntiles;
  uint64_t* hits;     // per probe row: match count << 32 | first payload (keys may repeat)
  uint32_t* pay;      // per probe row: its payload (no key repeats; aliases hits)
  uint64_t* hitmask;  // per 64 probe rows: which of them matched (no key repeats)
  int64_t* tile_cnt;
  int64_t* tile_off;
  uint32_t* out_idx;
  int32_t* out_pay;
  int64_t cap;
  int64_t* d_count;
  const int64_t* d_mult;  // largest number of build rows sharing one key
};

// Tiles belong to waves: wave tile t covers rows [t * chunk, (t + 1) * chunk),
// a multiple of 64 rows, processed in groups of 64 consecutive rows with lane
// l on row b0 + u * 64 + l, so key loads and record stores are contiguous per
// wave, and no step needs a workgroup barrier.
constexpr int kWaveRows = 64 * kProbe * 16;

__device__ __forceinline__ int64_t wave_tile() { return ((int64_t)blockIdx.x * kTPB + threadIdx.x) >> 6; }

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += (uint32_t)__shfl_xor((int)v, d, 64);
  return v;
}

// Probe pass: walks every row's chain once and records, per row, what the
// write pass needs, plus the wave tile's total.  When no key occurs twice in
// the table (the build's largest multiplicity is at most one) the record is
// the row's payload (4 bytes) and one bit of a per-64-row hit mask; otherwise
// it is the match count and first payload (count << 32 | payload).
//
// The walks are lane-independent.  A wave takes its tile in batches of
// kBatch rows; lane l owns rows l, l + 64, ... of a batch, whose keys it
// loads (coalesced across the wave) into its own LDS entries, and walks them
// one after another: when a row's walk ends the lane moves on to its next
// row at once, so every slot load of the wave serves a walk still in
// progress.  (A lockstep walk costs a wave as many slot loads as its longest
// chain, about seven at load 0.5 over 128 rows against a mean of 1.34; the
// probe's time follows the count of these scattered wave loads.)  A finished
// row's record replaces its key in LDS and the batch's records are stored
// coalesced.  Each lane touches only its own LDS entries, so no barrier is
// needed.  Keys and records are touched once, so they are loaded and stored
// non-temporally: they displace less of the table's hot lines from L2.
constexpr int kBatch = 512;
constexpr int kLaneRows = kBatch / 64;

template <class K>
__global__ __launch_bounds__(kTPB) void k_jp_probe(ProbeArgs a) {
  __shared__ uint64_t stage[kTPB / 64][kBatch];
  const int64_t t = wave_tile();
  if (t >= a.ntiles) return;
  const int64_t lo = t * a.chunk;
  const int64_t hi = min(a.n, lo + a.chunk);
  const int lane = threadIdx.x & 63;
  uint64_t* const st = stage[threadIdx.x >> 6] + lane;  // the lane's row j at st[j * 64]
  const bool first_only = *a.d_mult <= 1;
  const K* const pk = (const K*)a.pkey;
  uint32_t c = 0;
  for (int64_t b0 = lo; b0 < hi; b0 += kBatch) {
    const int64_t nb = min<int64_t>(kBatch, hi - b0);
    const int nv = lane < nb ? (int)((nb - lane + 63) >> 6) : 0;  // the lane's rows in the batch
    K kr[kLaneRows];  // rows past the tile read the tile's first row
#pragma unroll
    for (int j = 0; j < kLaneRows; ++j) {
      const int64_t r = b0 + (int64_t)j * 64 + lane;
      kr[j] = __builtin_nontemporal_load(pk + (r < hi ? r : lo));
    }
#pragma unroll
    for (int j = 0; j < kLaneRows; ++j) st[j * 64] = (uint64_t)(int64_t)kr[j];
    int j = 0;
    int64_t k = (int64_t)kr[0];
    uint64_t s = fmix64((uint64_t)k) & a.mask;
    uint32_t cnt = 0, first = 0;
    for (;;) {
      const bool act = j < nv;
      if (!__ballot(act)) break;
      // a lane without rows left reads slot 0 (one shared line)
      const uint4 sl = *(const uint4*)(a.slots + (act ? s : 0));  // (key lo, key hi, payload, used)
      // one 16-byte load: the compiler would otherwise split it into loads
      // sunk into the branches that read the fields, one wait each
      asm volatile("" ::"v"(sl.x), "v"(sl.y), "v"(sl.z), "v"(sl.w));
      if (act) {
        bool done = !sl.w;
        if (!done && (int64_t)(((uint64_t)sl.y << 32) | sl.x) == k) {
          if (cnt == 0) first = sl.z;
          ++cnt;
          done = first_only;
        }
        if (done) {
          st[j * 64] = ((uint64_t)cnt << 32) | first;
          c += cnt;
          if (++j < nv) {
            k = (int64_t)st[j * 64];
            s = fmix64((uint64_t)k) & a.mask;
            cnt = 0;
            first = 0;
          }
        } else {
          s = (s + 1) & a.mask;
        }
      }
    }
    if (first_only) {
#pragma unroll
      for (int j2 = 0; j2 < kLaneRows; ++j2) {
        const int64_t g = b0 + (int64_t)j2 * 64;  // 64-aligned: tiles and batches are multiples of 64 rows
        const uint64_t v = st[j2 * 64];
        const uint64_t m = __ballot(g + lane < hi && (v >> 32) != 0);
        if (g + lane < hi) __builtin_nontemporal_store((uint32_t)v, a.pay + g + lane);
        if (lane == 0 && g < hi) __builtin_nontemporal_store(m, a.hitmask + (g >> 6));
      }
    } else {
#pragma unroll
      for (int j2 = 0; j2 < kLaneRows; ++j2) {
        const int64_t r = b0 + (int64_t)j2 * 64 + lane;
        if (r < hi) __builtin_nontemporal_store(st[j2 * 64], a.hits + r);
      }
    }
  }
  c = wave_sum(c);
  if (lane == 0) a.tile_cnt[t] = c;
}

__global__ __launch_bounds__(kScanThreads) void k_jp_scan(ProbeArgs a) {
  __shared__ int64_t total;
  tile_offsets<kScanThreads>(a.tile_cnt, a.tile_off, a.ntiles, &total);
  __syncthreads();
  if (threadIdx.x == 0) {
    a.d_count[0] = total;
    a.d_count[1] = 0;
  }
}

// Write pass, one wave per tile: reads the recorded hits (no table access for
// rows with at most one match) and ranks the pairs in row order with a wave
// scan of the match counts and a running offset.  The pairs come out grouped
// by ascending probe row; a row with several matches walks its chain again,
// in the same order.
__global__ __launch_bounds__(kTPB) void k_jp_write(ProbeArgs a) {
  const int64_t t = wave_tile();
  if (t >= a.ntiles) return;
  const int64_t lo = t * a.chunk;
  const int64_t hi = min(a.n, lo + a.chunk);
  const int lane = threadIdx.x & 63;
  int64_t run = a.tile_off[t];
  if (*a.d_mult <= 1) {
    // one match at most per row: a 64-row group's pairs are ranked by its hit
    // mask; kGroups groups' masks and payloads are loaded together
    constexpr int kGroups = 4;
    const uint64_t below = (1ull << lane) - 1;
    for (int64_t b0 = lo; b0 < hi; b0 += 64 * kGroups) {
      uint64_t m[kGroups];
      uint32_t p[kGroups];
#pragma unroll
      for (int g = 0; g < kGroups; ++g) {
        const int64_t r = b0 + (int64_t)g * 64;
        m[g] = r < hi ? a.hitmask[r >> 6] : 0;
        p[g] = r + lane < hi ? __builtin_nontemporal_load(a.pay + r + lane) : 0;
      }
#pragma unroll
      for (int g = 0; g < kGroups; ++g) {
        if ((m[g] >> lane) & 1) {
          const int64_t o = run + __popcll(m[g] & below);
          if (o < a.cap) {
            a.out_idx[o] = (uint32_t)(b0 + (int64_t)g * 64 + lane);
            a.out_pay[o] = (int32_t)p[g];
          }
        }
        run += __popcll(m[g]);
      }
    }
    return;
  }
  for (int64_t b0 = lo; b0 < hi; b0 += 64 * kProbe) {
    int64_t idx[kProbe];
    uint64_t h[kProbe];
#pragma unroll
    for (int u = 0; u < kProbe; ++u) {
      idx[u] = b0 + (int64_t)u * 64 + lane;
      h[u] = idx[u] < hi ? a.hits[idx[u]] : 0;
    }
#pragma unroll
    for (int u = 0; u < kProbe; ++u) {
      const uint32_t cu = (uint32_t)(h[u] >> 32);
      uint32_t x = cu;  // inclusive scan over the wave
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = (uint32_t)__shfl_up((int)x, d, 64);
        if (lane >= d) x += y;
      }
      const int64_t o = run + (x - cu);
      run += (uint32_t)__shfl((int)x, 63, 64);
      if (cu == 0) continue;
      if (cu == 1) {
        if (o < a.cap) {
          a.out_idx[o] = (uint32_t)idx[u];
          a.out_pay[o] = (int32_t)(uint32_t)h[u];
        }
      } else {
        const int64_t k = load_i64(a.pkey, a.kdt, idx[u]);
        int64_t r = o;
        uint64_t sl_i = fmix64((uint64_t)k) & a.mask;
        for (uint64_t q = 0; q <= a.mask; ++q) {
          const JSlot sl = a.slots[sl_i];
          if (!sl.used) break;
          if (sl.key == k) {
            if (r < a.cap) {
              a.out_idx[r] = (uint32_t)idx[u];
              a.out_pay[r] = sl.pay;
            }
            ++r;
          }
          sl_i = (sl_i + 1) & a.mask;
        }
      }
    }
  }
}

__global__ void k_jp_empty(int64_t* d_count) {
  if (threadIdx.x == 0) {
    d_count[0] = 0;
    d_count[1] = 0;
  }
}

struct JpPlan {
  int64_t chunk;
  int ntiles;
};

JpPlan jp_plan(int64_t n) {
  JpPlan p;
  p.chunk = kWaveRows;
  while ((n + p.chunk - 1) / p.chunk > (1 << 20)) p.chunk *= 2;  // at most 2^20 wave tiles
  p.ntiles = (int)((n + p.chunk - 1) / p.chunk);
  return p;
}

size_t jp_workspace(int64_t n, ProbeArgs* a, void* base) {
  const JpPlan p = jp_plan(n);
  WsCarver c(base);
  int64_t* cnt = c.take<int64_t>(std::max(1, p.ntiles));
  int64_t* off = c.take<int64_t>(std::max(1, p.ntiles));
  uint64_t* hits = c.take<uint64_t>(std::max<int64_t>(1, n));
  uint64_t* mask = c.take<uint64_t>(std::max<int64_t>(1, (n + 63) / 64));
  if (a) {
    a->tile_cnt = cnt;
    a->tile_off = off;
    a->hits = hits;
    a->pay = (uint32_t*)hits;
    a->hitmask = mask;
  }
  return c.size();
}

}  // namespace
}  // namespace lms

using namespace lms;

extern "C" int lms_join_build(const lms_batch* tbl, int32_t key_col, int32_t payload_col, lms_join_table** out,
                              lms_stream stream) {
  if (!tbl || !out) return set_error(LMS_EINVAL, "table/out is NULL");
  *out = nullptr;
  if (tbl->ncols <= 0 || !tbl->cols) return set_error(LMS_EINVAL, "table has no columns");
  if (key_col < 0 || key_col >= tbl->ncols) return set_error(LMS_EINVAL, "key column %d out of range", key_col);
  if (payload_col < 0 || payload_col >= tbl->ncols)
    return set_error(LMS_EINVAL, "payload column %d out of range", payload_col);
  const int kdt = tbl->cols[key_col].dtype;
  if (kdt != LMS_I32 && kdt != LMS_I64) return set_error(LMS_EINVAL, "join key must be integer");
  if (tbl->cols[payload_col].dtype != LMS_I32) return set_error(LMS_EINVAL, "payload column must be int32");
  if (tbl->nrows < 0 || tbl->nrows >= (int64_t(1) << 31)) return set_error(LMS_EINVAL, "build side must have < 2^31 rows");
  if (tbl->nrows > 0 && (!tbl->cols[key_col].data || !tbl->cols[payload_col].data))
    return set_error(LMS_EINVAL, "table column data is NULL");
  uint64_t nslots = 64;
  while (nslots < 2 * (uint64_t)tbl->nrows) nslots <<= 1;
  lms_join_table* t = new lms_join_table{};
  t->mask = nslots - 1;
  t->nbuild = tbl->nrows;
  t->mult_cache = -1;
  int rc = check_hip(hipMalloc(&t->slots, nslots * sizeof(JSlot)), "hipMalloc join table");
  if (!rc) rc = check_hip(hipMalloc(&t->d_mult, sizeof(int64_t)), "hipMalloc join counter");
  if (!rc) rc = check_hip(hipEventCreateWithFlags(&t->built, hipEventDisableTiming), "hipEventCreate");
  if (rc) {
    if (t->slots) hipFree(t->slots);
    if (t->d_mult) hipFree(t->d_mult);
    delete t;
    return rc == LMS_EHIP ? LMS_ENOMEM : rc;
  }
  hipStream_t st = (hipStream_t)stream;
  LMS_LAUNCH("k_jb_clear", k_jb_clear, dim3((unsigned)((nslots + 255) / 256)), dim3(256), 0, st, t->slots, nslots,
                     t->d_mult);
  if (tbl->nrows > 0) {
    LMS_LAUNCH("k_jb_insert", k_jb_insert, dim3((unsigned)((tbl->nrows + 255) / 256)), dim3(256), 0, st, t->slots, t->mask,
                       (const void*)tbl->cols[key_col].data, kdt, (const int32_t*)tbl->cols[payload_col].data,
                       tbl->nrows);
    LMS_LAUNCH("k_jb_mult", k_jb_mult, dim3((unsigned)((nslots + kTPB - 1) / kTPB)), dim3(kTPB), 0, st, t->slots, t->mask,
                       t->d_mult);
  }
  rc = check_hip(hipGetLastError(), "join build launch");
  if (!rc) rc = check_hip(hipEventRecord(t->built, st), "hipEventRecord");
  if (rc) {
    lms_join_free(t);
    return rc;
  }
  *out = t;
  return LMS_OK;
}

extern "C" int64_t lms_join_max_mult(lms_join_table* t) {
  if (!t) return set_error(LMS_EINVAL, "table is NULL");
  if (t->mult_cache >= 0) return t->mult_cache;
  int rc = check_hip(hipEventSynchronize(t->built), "hipEventSynchronize");
  if (rc) return rc;
  int64_t m = 0;
  rc = check_hip(hipMemcpy(&m, t->d_mult, sizeof m, hipMemcpyDeviceToHost), "hipMemcpy");
  if (rc) return rc;
  t->mult_cache = m;
  return m;
}

extern "C" int64_t lms_join_build_rows(const lms_join_table* t) { return t ? t->nbuild : LMS_EINVAL; }

extern "C" void lms_join_free(lms_join_table* t) {
  if (!t) return;
  hipEventSynchronize(t->built);
  hipFree(t->slots);
  hipFree(t->d_mult);
  hipEventDestroy(t->built);
  delete t;
}

extern "C" size_t lms_hash_join_workspace(int64_t nprobe) {
  return nprobe < 0 ? 0 : jp_workspace(nprobe, nullptr, nullptr);
}

extern "C" int lms_hash_join(const lms_join_table* t, const lms_batch* probe, int32_t key_col, uint32_t* out_probe_idx,
                             int32_t* out_payload, int64_t cap, int64_t* d_count, void* workspace, size_t ws_bytes,
                             lms_stream stream) {
  if (!t || !probe || !d_count) return set_error(LMS_EINVAL, "table/probe/d_count is NULL");
  if (probe->nrows < 0 || probe->nrows >= (int64_t(1) << 32))
    return set_error(LMS_EINVAL, "probe batch must have < 2^32 rows");
  if (key_col < 0 || key_col >= probe->ncols || !probe->cols)
    return set_error(LMS_EINVAL, "probe key column %d out of range", key_col);
  const int kdt = probe->cols[key_col].dtype;
  if (kdt != LMS_I32 && kdt != LMS_I64) return set_error(LMS_EINVAL, "probe key must be integer");
  if (probe->nrows > 0 && !probe->cols[key_col].data) return set_error(LMS_EINVAL, "probe key data is NULL");
  if (cap < 0) return set_error(LMS_EINVAL, "negative capacity");
  if (cap > 0 && (!out_probe_idx || !out_payload)) return set_error(LMS_EINVAL, "output arrays are NULL");
  const size_t need = jp_workspace(probe->nrows, nullptr, nullptr);
  if (!workspace || ws_bytes < need)
    return set_error(LMS_ENOMEM, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes, need);
  ProbeArgs a{};
  jp_workspace(probe->nrows, &a, workspace);
  const JpPlan p = jp_plan(probe->nrows);
  a.slots = t->slots;
  a.mask = t->mask;
  a.pkey = probe->cols[key_col].data;
  a.kdt = kdt;
  a.n = probe->nrows;
  a.chunk = p.chunk;
  a.ntiles = p.ntiles;
  a.out_idx = out_probe_idx;
  a.out_pay = out_payload;
  a.cap = cap;
  a.d_count = d_count;
  a.d_mult = t->d_mult;
  hipStream_t st = (hipStream_t)stream;
  // the build may run on another stream: order this probe after it
  int rc = check_hip(hipStreamWaitEvent(st, t->built, 0), "hipStreamWaitEvent");
  if (rc) return rc;
  if (probe->nrows == 0) {
    LMS_LAUNCH("k_jp_empty", k_jp_empty, dim3(1), dim3(64), 0, st, d_count);
  } else {
    const unsigned wgs = (unsigned)((p.ntiles + kTPB / 64 - 1) / (kTPB / 64));  // one wave per tile
    if (kdt == LMS_I32)
      LMS_LAUNCH("k_jp_probe", k_jp_probe<int32_t>, dim3(wgs), dim3(kTPB), 0, st, a);
    else
      LMS_LAUNCH("k_jp_probe", k_jp_probe<int64_t>, dim3(wgs), dim3(kTPB), 0, st, a);
    LMS_LAUNCH("k_jp_scan", k_jp_scan, dim3(1), dim3(kScanThreads), 0, st, a);
    LMS_LAUNCH("k_jp_write", k_jp_write, dim3(wgs), dim3(kTPB), 0, st, a);
  }
  return check_hip(hipGetLastError(), "hash_join launch");
}
