// The cell sort of the particles: the unique (cell key, id) order, the row index of the
// sorted stream and the payloads that travel with it, in four steps.
//
//   1. row_count:  particles per row segment (item, ix, iy and the top bits of iz: a row or
//                  a part of it, cell_sort_split) = key >> (log2(nm) - split), with one
//                  atomic per distinct segment per wavefront.
//   2. row_scan:   exclusive scan of the counts -> row_start (the row index the paints and
//                  gathers use) and a cursor per row.
//   3. bucket:     every particle id into its row's range, at a slot taken from the row's
//                  cursor (the order inside a row depends on the timing of the atomics).
//   4. row sort:   each row's entries sorted by the 64-bit composite (iz << 32 | id), which
//                  is unique per particle, so the result is the (key, id) order whatever the
//                  bucket order was: a wavefront sorts rows of up to 256 entries in registers
//                  (bitonic network across lanes), a workgroup rows of up to 4096 in LDS, and
//                  a workgroup runs a stable LSD radix sort in global memory for larger rows
//                  (which only occur in very dense layouts). Every sorted entry is written
//                  with its payload (gathered by id) and its inverse permutation entry.
//
// Compulsory traffic: the id-order keys read twice (count, bucket), one id written and read
// per particle in the buckets, the sorted keys, ids and payload written; no pass over
// 8-bit digits of the whole key array.
#include "pmr_internal.h"

namespace pmr {
namespace {

constexpr int TB = 256;
constexpr int WAVE_ROW_MAX = 256;    // tier 1: one wavefront, 4 entries per lane
constexpr int BLOCK_ROW_MAX = 4096;  // tier 2: one workgroup, 16 entries per thread in LDS
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = TB * SCAN_ITEMS;  // counts per scan block

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ uint64_t lanes_below() {
  const int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// The value of lane (lane ^ J). Distances 1 and 2 are DPP quad permutations and 4 and 8
// DPP row shifts (row_shl:J reads lane + J, row_shr:J lane - J, inside a row of 16 lanes,
// where lane ^ J stays for these J): VALU moves with no LDS round trip. The moves carry no
// old operand (the bound control reads 0 out of range, and the shift whose source is out of
// range is the one not selected), so no register is cleared before them. 16 and 32 use the
// row swaps of gfx950 on two copies of the value: permlane16_swap leaves the first copy
// with rows (0, 0, 2, 2) and the second with (1, 1, 3, 3) of the original, permlane32_swap
// the halves (lo, lo) and (hi, hi), so each lane picks the copy that holds its partner.
template <int J>
__device__ __forceinline__ uint32_t xor_lane(uint32_t v) {
  if constexpr (J == 1) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, true);  // [1,0,3,2]
  } else if constexpr (J == 2) {
    return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, true);  // [2,3,0,1]
  } else if constexpr (J == 4 || J == 8) {
    const uint32_t up = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x100 + J, 0xF, 0xF, true);
    const uint32_t dn = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x110 + J, 0xF, 0xF, true);
    return (lane_id() & J) ? dn : up;
  } else if constexpr (J == 16) {
    const auto p = __builtin_amdgcn_permlane16_swap(v, v, false, false);
    return (lane_id() & 16) ? p[0] : p[1];
  } else {
    const auto p = __builtin_amdgcn_permlane32_swap(v, v, false, false);
    return (lane_id() & 32) ? p[0] : p[1];
  }
}

template <int J>
__device__ __forceinline__ uint64_t xor_lane64(uint64_t v) {
  const uint32_t lo = xor_lane<J>((uint32_t)v);
  const uint32_t hi = xor_lane<J>((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

__global__ void fill_u32_kernel(uint32_t* __restrict__ p, size_t n, uint32_t v) {
  for (size_t i = (size_t)blockIdx.x * TB + threadIdx.x; i < n; i += (size_t)gridDim.x * TB)
    p[i] = v;
}

// ---------------------------------------------------------------- 1. counts
// The 64 (row, lane) pairs of a wavefront sorted by a bitonic network across lanes, so that
// equal rows form runs: the first lane of each run then issues one atomic for the whole run,
// all runs at once (instead of one round trip per distinct row). Rows must be <= 2^25 (the
// caller checks), so that no entry equals the end marker ~0 that lanes past the end carry.
template <int K, int J>
__device__ __forceinline__ void sort64_stage(uint32_t& v) {
  const int lane = lane_id();
  const uint32_t o = xor_lane<J>(v);
  const bool keep_min = ((lane & J) == 0) == ((lane & K) == 0);
  v = keep_min ? (v < o ? v : o) : (v < o ? o : v);
  if constexpr (J > 1) sort64_stage<K, J / 2>(v);
}

template <int K>
__device__ __forceinline__ void sort64_level(uint32_t& v) {
  sort64_stage<K, K / 2>(v);
  if constexpr (K < 64) sort64_level<2 * K>(v);
}

// Ascending bitonic sort of one value per lane across the 64 lanes.
__device__ __forceinline__ uint32_t wave_sort64(uint32_t v) {
  sort64_level<2>(v);
  return v;
}

// Runs of equal rows among the sorted (row << 6 | lane) values: for each lane the row, the
// first lane of its run and the run's length (valid only for real entries).
struct WaveRuns {
  uint32_t row;
  int head, len;
  bool ok;
};

__device__ __forceinline__ WaveRuns wave_runs(uint32_t sorted) {
  const int lane = lane_id();
  WaveRuns w;
  w.ok = sorted != ~0u;
  w.row = sorted >> 6;
  const uint32_t prev = __shfl_up(w.row, 1, 64);
  const bool head = w.ok && (lane == 0 || prev != w.row);
  const uint64_t heads = __ballot(head);
  const uint64_t valid = __ballot(w.ok);
  const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);  // lanes 0..lane
  w.head = 63 - __clzll((long long)(heads & upto));
  const uint64_t after = heads & ~upto;  // heads above this lane
  const int end = after ? __ffsll((unsigned long long)after) - 1 : __popcll(valid);
  w.len = end - w.head;
  return w;
}

// Particles are visited in `order` (a permutation of the ids, nullable: id order). The
// previous step's sorted order groups particles by their old cell, and a particle moves
// about a cell per step, so a wavefront of it falls in one or two new rows.
__device__ __forceinline__ uint32_t visit(const uint32_t* __restrict__ order, int g) {
  return order ? order[g] : (uint32_t)g;
}

// Groups of 64 particles per wavefront and launch (each thread holds one particle of each
// group, loaded together so that the loads of the groups overlap). Two measured 1.5% faster
// for the sort than four at 256^3 on 512^3 and the same at 128^3 x 4; eight was slower.
constexpr int GROUPS = 2;

__device__ __forceinline__ int group_base(int q) {
  return ((blockIdx.x * (TB / 64) + (threadIdx.x >> 6)) * GROUPS + q) * 64;
}

__global__ __launch_bounds__(TB) void row_count_kernel(const uint32_t* __restrict__ keys,
                                                       const uint32_t* __restrict__ order, int n,
                                                       int shift, uint32_t* __restrict__ cnt) {
  const int lane = lane_id();
  uint32_t id[GROUPS], v[GROUPS];
#pragma unroll
  for (int q = 0; q < GROUPS; ++q) {
    const int g = group_base(q) + lane;
    id[q] = g < n ? visit(order, g) : 0u;
  }
#pragma unroll
  for (int q = 0; q < GROUPS; ++q) {
    const int g = group_base(q) + lane;
    v[q] = g < n ? ((keys[id[q]] >> shift) << 6) | (uint32_t)lane : ~0u;
  }
#pragma unroll
  for (int q = 0; q < GROUPS; ++q) {
    const WaveRuns w = wave_runs(wave_sort64(v[q]));
    if (w.ok && w.head == lane) atomicAdd(&cnt[w.row], (uint32_t)w.len);
  }
}

// The same with one round trip per distinct row (any number of rows).
__global__ __launch_bounds__(TB) void row_count_loop_kernel(const uint32_t* __restrict__ keys,
                                                            const uint32_t* __restrict__ order,
                                                            int n, int shift,
                                                            uint32_t* __restrict__ cnt) {
  const int g = blockIdx.x * TB + threadIdx.x;
  const bool ok = g < n;
  const uint32_t r = ok ? keys[visit(order, g)] >> shift : 0u;
  uint64_t todo = __ballot(ok);
  while (todo) {
    const int leader = __ffsll((unsigned long long)todo) - 1;
    const uint32_t rl = __shfl(r, leader, 64);
    const uint64_t same = __ballot(ok && r == rl);
    if (lane_id() == leader) atomicAdd(&cnt[rl], (uint32_t)__popcll(same));
    todo &= ~same;
  }
}

// ---------------------------------------------------------------- 2. scan
// Inclusive scan over the block of one value per thread (wavefront shuffles, then the
// wavefront totals); returns the inclusive prefix and the block total.
__device__ __forceinline__ uint32_t block_inclusive_scan(uint32_t v, uint32_t* wsum,
                                                         uint32_t* total) {
  const int lane = lane_id(), w = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  uint32_t pre = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < TB / 64; ++i) {
    const uint32_t s = wsum[i];
    if (i < w) pre += s;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return pre + x;
}

// partial[b] = sum of counts of scan block b
__global__ __launch_bounds__(TB) void scan_reduce_kernel(const uint32_t* __restrict__ cnt,
                                                         size_t rows,
                                                         uint32_t* __restrict__ partial) {
  __shared__ uint32_t wsum[TB / 64];
  const size_t base = (size_t)blockIdx.x * SCAN_TILE + (size_t)threadIdx.x * SCAN_ITEMS;
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) s += base + i < rows ? cnt[base + i] : 0u;
  uint32_t tot;
  block_inclusive_scan(s, wsum, &tot);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// exclusive scan of the block partials in place (one workgroup, any number of blocks)
__global__ __launch_bounds__(TB) void scan_partials_kernel(uint32_t* __restrict__ partial,
                                                           int nb) {
  __shared__ uint32_t wsum[TB / 64];
  uint32_t carry = 0;
  for (int b0 = 0; b0 < nb; b0 += TB) {
    const int b = b0 + threadIdx.x;
    const uint32_t v = b < nb ? partial[b] : 0u;
    uint32_t tot;
    const uint32_t inc = block_inclusive_scan(v, wsum, &tot);
    if (b < nb) partial[b] = carry + inc - v;
    carry += tot;
  }
}

// start[r] = exclusive prefix of the counts of the segments; cursor[r] = start[r];
// start[rows] = n (the total); the row index of the caller gets the start of every
// (1 << split)-th segment (the first segment of each row).
__global__ __launch_bounds__(TB) void scan_write_kernel(const uint32_t* __restrict__ cnt,
                                                        size_t rows,
                                                        const uint32_t* __restrict__ partial,
                                                        uint32_t n,
                                                        uint32_t* __restrict__ row_start,
                                                        uint32_t* __restrict__ cursor,
                                                        uint32_t* __restrict__ seg_start,
                                                        int split) {
  __shared__ uint32_t wsum[TB / 64];
  const size_t base = (size_t)blockIdx.x * SCAN_TILE + (size_t)threadIdx.x * SCAN_ITEMS;
  uint32_t v[SCAN_ITEMS];
  uint32_t s = 0;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    v[i] = base + i < rows ? cnt[base + i] : 0u;
    s += v[i];
  }
  uint32_t tot;
  uint32_t run = partial[blockIdx.x] + block_inclusive_scan(s, wsum, &tot) - s;
#pragma unroll
  for (int i = 0; i < SCAN_ITEMS; ++i) {
    const size_t r = base + i;
    if (r < rows) {
      seg_start[r] = run;
      cursor[r] = run;
      if ((r & (((size_t)1 << split) - 1)) == 0) row_start[r >> split] = run;
    }
    run += v[i];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    seg_start[rows] = n;
    row_start[rows >> split] = n;
  }
}

// ---------------------------------------------------------------- 3. buckets
__global__ __launch_bounds__(TB) void bucket_kernel(const uint32_t* __restrict__ keys,
                                                    const uint32_t* __restrict__ order, int n,
                                                    int shift, uint32_t* __restrict__ cursor,
                                                    uint32_t* __restrict__ bucket) {
  const int lane = lane_id();
  uint32_t id[GROUPS], v[GROUPS];
#pragma unroll
  for (int q = 0; q < GROUPS; ++q) {
    const int g = group_base(q) + lane;
    id[q] = g < n ? visit(order, g) : 0u;
  }
#pragma unroll
  for (int q = 0; q < GROUPS; ++q) {
    const int g = group_base(q) + lane;
    v[q] = g < n ? ((keys[id[q]] >> shift) << 6) | (uint32_t)lane : ~0u;
  }
#pragma unroll
  for (int q = 0; q < GROUPS; ++q) {
    const uint32_t sorted = wave_sort64(v[q]);
    const WaveRuns w = wave_runs(sorted);
    uint32_t base = 0;
    if (w.ok && w.head == lane) base = atomicAdd(&cursor[w.row], (uint32_t)w.len);
    base = __shfl(base, w.ok ? w.head : lane, 64);
    const uint32_t src_id = __shfl(id[q], (int)(sorted & 63u), 64);
    if (w.ok) bucket[base + (uint32_t)(lane - w.head)] = src_id;
  }
}

__global__ __launch_bounds__(TB) void bucket_loop_kernel(const uint32_t* __restrict__ keys,
                                                         const uint32_t* __restrict__ order,
                                                         int n, int shift,
                                                         uint32_t* __restrict__ cursor,
                                                         uint32_t* __restrict__ bucket) {
  const int g = blockIdx.x * TB + threadIdx.x;
  const bool ok = g < n;
  const uint32_t id = ok ? visit(order, g) : 0u;
  const uint32_t r = ok ? keys[id] >> shift : 0u;
  uint64_t todo = __ballot(ok);
  uint32_t pos = 0;
  while (todo) {
    const int leader = __ffsll((unsigned long long)todo) - 1;
    const uint32_t rl = __shfl(r, leader, 64);
    const bool mine = ok && r == rl;
    const uint64_t same = __ballot(mine);
    uint32_t base = 0;
    if (lane_id() == leader) base = atomicAdd(&cursor[rl], (uint32_t)__popcll(same));
    base = __shfl(base, leader, 64);
    if (mine) pos = base + (uint32_t)__popcll(same & lanes_below());
    todo &= ~same;
  }
  if (ok) bucket[pos] = id;
}

// ---------------------------------------------------------------- 4. row sorts
struct RowSortArgs {
  const uint32_t* keys;       // id-order keys
  const uint32_t* row_start;  // [rows + 1]
  const uint32_t* bucket;     // ids bucketed by row
  uint32_t* keys_sorted;
  uint32_t* ids_sorted;
  const Vec3* pay_in;  // nullable
  Vec3* pay_out;
  uint32_t* inv;       // nullable
  uint32_t* tmp_hi;    // global radix scratch [n] x 2 (rows beyond the LDS tier)
  uint32_t* tmp_lo;
  int shift;
  uint32_t zmask;      // nm - 1
  int idbits;          // bits of the largest id (32-bit composites: iz << idbits | id)
  size_t rows;
  int block_rows;      // rows a workgroup of the long-row tiers tests per step (<= TB)
};

// Composite sort value of a particle within its row: (iz, id) as iz << 32 | id in 64 bits,
// or iz << idbits | id in 32 bits where the two fit (the order is the same).
template <typename T>
__device__ __forceinline__ T composite_t(const RowSortArgs& a, uint32_t id) {
  if constexpr (sizeof(T) == 8)
    return ((uint64_t)(a.keys[id] & a.zmask) << 32) | id;
  else
    return ((a.keys[id] & a.zmask) << a.idbits) | id;
}

// Writes one sorted entry at sorted position pos of row `row`, with its payload
// (non-temporal: read once, by the paint after the sort) and inverse permutation entry.
// (A separate streaming pass over the sorted ids for these measured no faster at 256^3 on
// 512^3 and 2% slower for the sort at 128^3 x 4: the gather by id costs the same in either.)
template <typename T>
__device__ __forceinline__ void emit_t(const RowSortArgs& a, uint32_t row, uint32_t pos, T v) {
  uint32_t iz, id;
  if constexpr (sizeof(T) == 8) {
    iz = (uint32_t)(v >> 32);
    id = (uint32_t)v;
  } else {
    iz = v >> a.idbits;
    id = v & ((1u << a.idbits) - 1u);
  }
  a.keys_sorted[pos] = (row << a.shift) | iz;
  a.ids_sorted[pos] = id;
  if (a.pay_out) {
    const Vec3 p = a.pay_in[id];
    __builtin_nontemporal_store(p.x, &a.pay_out[pos].x);
    __builtin_nontemporal_store(p.y, &a.pay_out[pos].y);
    __builtin_nontemporal_store(p.z, &a.pay_out[pos].z);
  }
  if (a.inv) a.inv[id] = pos;
}

__device__ __forceinline__ void emit(const RowSortArgs& a, uint32_t row, uint32_t pos, uint64_t v) {
  emit_t<uint64_t>(a, row, pos, v);
}

template <typename T, int J>
__device__ __forceinline__ T xor_lane_t(T v) {
  if constexpr (sizeof(T) == 8)
    return xor_lane64<J>(v);
  else
    return xor_lane<J>(v);
}

// Bitonic sort of 64 K values, element e * 64 + lane in v[e], ascending: level k merges
// runs of k, stage j compares elements j apart (across lanes for j < 64, across the
// registers of one lane for j >= 64).
template <typename T, int K, int k, int j>
__device__ __forceinline__ void bitonic_stage(T (&v)[K]) {
  const int lane = lane_id();
  if constexpr (j >= 64) {
    constexpr int je = j >> 6;
#pragma unroll
    for (int e = 0; e < K; ++e) {
      if ((e & je) == 0) {
        const int p = e | je;
        const bool up = ((e * 64 + lane) & k) == 0;
        const T x = v[e], y = v[p];
        const bool sw = (x > y) == up;
        v[e] = sw ? y : x;
        v[p] = sw ? x : y;
      }
    }
  } else {
    const bool lower = (lane & j) == 0;
#pragma unroll
    for (int e = 0; e < K; ++e) {
      const T o = xor_lane_t<T, j>(v[e]);
      const bool up = ((e * 64 + lane) & k) == 0;
      v[e] = (lower == up) ? (v[e] < o ? v[e] : o) : (v[e] < o ? o : v[e]);
    }
  }
  if constexpr (j > 1) bitonic_stage<T, K, k, j / 2>(v);
}

template <typename T, int K, int k>
__device__ __forceinline__ void bitonic_level(T (&v)[K]) {
  bitonic_stage<T, K, k, k / 2>(v);
  if constexpr (k < 64 * K) bitonic_level<T, K, 2 * k>(v);
}

template <typename T, int K>
__device__ __forceinline__ void wave_bitonic(T (&v)[K]) {
  bitonic_level<T, K, 2>(v);
}

// Tier 1: each wavefront takes two rows at a time (r and r + W for W wavefronts), loading
// both before sorting either, so that their dependent loads (row start, bucket, key
// gather) overlap; rows of 1..256 entries are sorted here. (Two rows per step measured
// 2-3% faster for the sort than one or four, and eight 13% slower: more rows in flight
// cost resident waves.)
constexpr int WAVE_ROWS = 2;

template <typename T>
__global__ __launch_bounds__(TB) void row_sort_wave_kernel(RowSortArgs a) {
  constexpr T PADT = (T)~(T)0;  // sorts after (or ties with) every real entry
  const size_t waves = (size_t)gridDim.x * (TB / 64);
  const int lane = lane_id();
  for (size_t r0 = (size_t)blockIdx.x * (TB / 64) + (threadIdx.x >> 6); r0 < a.rows;
       r0 += WAVE_ROWS * waves) {
    uint32_t start[WAVE_ROWS], cnt[WAVE_ROWS];
#pragma unroll
    for (int q = 0; q < WAVE_ROWS; ++q) {
      const size_t r = r0 + q * waves;
      start[q] = r < a.rows ? a.row_start[r] : 0u;
      cnt[q] = r < a.rows ? a.row_start[r + 1] - start[q] : 0u;
      if (cnt[q] > WAVE_ROW_MAX) cnt[q] = 0;  // the workgroup tiers take it
    }
    uint32_t id[WAVE_ROWS][4];
#pragma unroll
    for (int q = 0; q < WAVE_ROWS; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const uint32_t i = e * 64 + lane;
        id[q][e] = i < cnt[q] ? a.bucket[start[q] + i] : 0u;
      }
    T v[WAVE_ROWS][4];
#pragma unroll
    for (int q = 0; q < WAVE_ROWS; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const uint32_t i = e * 64 + lane;
        v[q][e] = i < cnt[q] ? composite_t<T>(a, id[q][e]) : PADT;
      }
#pragma unroll
    for (int q = 0; q < WAVE_ROWS; ++q) {
      if (cnt[q] == 0) continue;
      const uint32_t row = (uint32_t)(r0 + q * waves);
      if (cnt[q] <= 64) {
        T w1[1] = {v[q][0]};
        wave_bitonic<T, 1>(w1);
        if (lane < (int)cnt[q]) emit_t<T>(a, row, start[q] + lane, w1[0]);
      } else if (cnt[q] <= 128) {
        T w2[2] = {v[q][0], v[q][1]};
        wave_bitonic<T, 2>(w2);
#pragma unroll
        for (int e = 0; e < 2; ++e)
          if ((uint32_t)(e * 64 + lane) < cnt[q]) emit_t<T>(a, row, start[q] + e * 64 + lane, w2[e]);
      } else {
        wave_bitonic<T, 4>(v[q]);
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if ((uint32_t)(e * 64 + lane) < cnt[q])
            emit_t<T>(a, row, start[q] + e * 64 + lane, v[q][e]);
      }
    }
  }
}

// Stable scatter of one LSD radix pass over 8 bits of the composite held as (hi, lo) pairs,
// src -> dst within one row's range, by one workgroup, chunk by chunk in order.
__device__ void block_radix_pass(const uint32_t* shi, const uint32_t* slo, uint32_t* dhi,
                                 uint32_t* dlo, uint32_t c, int bit, uint32_t* base,
                                 uint32_t (*wcnt)[256]) {
  const int t = threadIdx.x, lane = lane_id(), w = t >> 6;
  auto digit = [&](uint32_t hi, uint32_t lo) -> uint32_t {
    return bit >= 32 ? (hi >> (bit - 32)) & 255u : (lo >> bit) & 255u;
  };
  // histogram -> exclusive digit offsets
  base[t] = 0;
  __syncthreads();
  for (uint32_t i = t; i < c; i += TB) atomicAdd(&base[digit(shi[i], slo[i])], 1u);
  __syncthreads();
  {
    __shared__ uint32_t wsum[TB / 64];
    const uint32_t v = base[t];
    uint32_t tot;
    const uint32_t inc = block_inclusive_scan(v, wsum, &tot);
    base[t] = inc - v;
  }
  __syncthreads();
  for (uint32_t c0 = 0; c0 < c; c0 += TB) {
    const uint32_t i = c0 + t;
    const bool ok = i < c;
    const uint32_t hi = ok ? shi[i] : 0u, lo = ok ? slo[i] : 0u;
    const uint32_t d = ok ? digit(hi, lo) : 0u;
    for (int q = 0; q < TB / 64; ++q) wcnt[q][t] = 0;
    __syncthreads();
    uint64_t m = __ballot(ok);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool on = (d >> b) & 1u;
      const uint64_t bal = __ballot(on);
      m &= on ? bal : ~bal;
    }
    const uint32_t rank = (uint32_t)__popcll(m & lanes_below());
    if (ok && rank == 0) wcnt[w][d] = (uint32_t)__popcll(m);
    __syncthreads();
    if (ok) {
      uint32_t pos = base[d] + rank;
      for (int q = 0; q < w; ++q) pos += wcnt[q][d];
      dhi[pos] = hi;
      dlo[pos] = lo;
    }
    __syncthreads();
    uint32_t add = 0;
    for (int q = 0; q < TB / 64; ++q) add += wcnt[q][t];
    base[t] += add;
    __syncthreads();
  }
}

// Tier 2 (rows of 257..4096 entries: bitonic sort in LDS) and tier 3 (larger rows: stable
// LSD radix passes in global memory over the digits that vary in the row). A workgroup
// takes block_rows consecutive rows at a time (blocks strided over the row range); its
// threads test those rows' lengths together and the workgroup then sorts the long ones one
// after the other (rows are independent, so the order in which they are done does not
// matter). block_rows is chosen so that every resident workgroup gets rows to test.
template <typename T>
__global__ __launch_bounds__(TB) void row_sort_block_kernel(RowSortArgs a) {
  constexpr T PADT = (T)~(T)0;
  __shared__ T s[BLOCK_ROW_MAX];
  __shared__ uint32_t base[256];
  __shared__ uint32_t wcnt[TB / 64][256];
  __shared__ uint32_t red[2][TB / 64];
  __shared__ uint32_t found[TB];
  __shared__ int nfound;
  const int t = threadIdx.x;
  const size_t br = (size_t)a.block_rows;
  for (size_t r0 = (size_t)blockIdx.x * br; r0 < a.rows; r0 += (size_t)gridDim.x * br) {
    if (t == 0) nfound = 0;
    __syncthreads();
    if ((size_t)t < br && r0 + t < a.rows &&
        a.row_start[r0 + t + 1] - a.row_start[r0 + t] > WAVE_ROW_MAX)
      found[atomicAdd(&nfound, 1)] = (uint32_t)t;
    __syncthreads();
    const int nf = nfound;
    for (int f = 0; f < nf; ++f) {
      const size_t r = r0 + found[f];
      const uint32_t start = a.row_start[r];
      const uint32_t c = a.row_start[r + 1] - start;
      const uint32_t row = (uint32_t)r;
      if (c <= BLOCK_ROW_MAX) {
        uint32_t p2 = 512;
        while (p2 < c) p2 <<= 1;
        for (uint32_t i = t; i < p2; i += TB)
          s[i] = i < c ? composite_t<T>(a, a.bucket[start + i]) : PADT;
        __syncthreads();
        for (uint32_t k = 2; k <= p2; k <<= 1) {
          for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t q = t; q < p2 / 2; q += TB) {
              const uint32_t i = ((q & ~(j - 1)) << 1) | (q & (j - 1));
              const uint32_t p = i | j;
              const bool up = (i & k) == 0;
              const T x = s[i], y = s[p];
              if ((x > y) == up) {
                s[i] = y;
                s[p] = x;
              }
            }
            __syncthreads();
          }
        }
        for (uint32_t i = t; i < c; i += TB) emit_t<T>(a, row, start + i, s[i]);
        __syncthreads();
        continue;
      }
      // tier 3: (hi, lo) = (iz, id) pairs; A = the row's range of the sorted outputs, B = the
      // radix scratch
      uint32_t* ahi = a.keys_sorted + start;
      uint32_t* alo = a.ids_sorted + start;
      uint32_t* bhi = a.tmp_hi + start;
      uint32_t* blo = a.tmp_lo + start;
      uint32_t orv[2] = {0u, 0u}, andv[2] = {~0u, ~0u};
      for (uint32_t i = t; i < c; i += TB) {
        const uint32_t id = a.bucket[start + i];
        const uint32_t hi = a.keys[id] & a.zmask;
        ahi[i] = hi;
        alo[i] = id;
        orv[0] |= hi;
        andv[0] &= hi;
        orv[1] |= id;
        andv[1] &= id;
      }
      // bits that vary across the row (passes over constant digits are skipped)
      uint32_t var[2];
      for (int h = 0; h < 2; ++h) {
        uint32_t o = orv[h], n = andv[h];
  #pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
          o |= __shfl_xor(o, d, 64);
          n &= __shfl_xor(n, d, 64);
        }
        if (lane_id() == 0) {
          red[0][t >> 6] = o;
          red[1][t >> 6] = n;
        }
        __syncthreads();
        o = 0u;
        n = ~0u;
        for (int q = 0; q < TB / 64; ++q) {
          o |= red[0][q];
          n &= red[1][q];
        }
        var[h] = o ^ n;
        __syncthreads();
      }
      bool in_a = true;
      for (int bit = 0; bit < 64; bit += 8) {
        const uint32_t vm = bit >= 32 ? var[0] >> (bit - 32) : var[1] >> bit;
        if ((vm & 255u) == 0) continue;
        __syncthreads();  // the previous pass's writes
        if (in_a)
          block_radix_pass(ahi, alo, bhi, blo, c, bit, base, wcnt);
        else
          block_radix_pass(bhi, blo, ahi, alo, c, bit, base, wcnt);
        in_a = !in_a;
      }
      __syncthreads();
      const uint32_t* fhi = in_a ? ahi : bhi;
      const uint32_t* flo = in_a ? alo : blo;
      // each thread reads and rewrites only its own indices of A (in place when the last pass
      // landed there)
      for (uint32_t i = t; i < c; i += TB)
        emit(a, row, start + i, ((uint64_t)fhi[i] << 32) | flo[i]);
      __syncthreads();
    }
    __syncthreads();  // every thread has read nfound before it is reset
  }
}

int grid_for(size_t n, int per_block) {
  const size_t b = (n + per_block - 1) / per_block;
  return (int)(b < 1 ? 1 : b);
}

}  // namespace

// Row segments: the sort works on segments of 2^split cells of a row (split low bits of iz
// moved into the segment number), chosen so that the (iz, id) composite of a segment fits
// 32 bits and a segment holds 64 particles or fewer on average (so the wavefront tier
// takes nearly every segment).
int cell_sort_split(int n, size_t rows, int shift) {
  int idbits = 0;
  while (idbits < 32 && ((size_t)1 << idbits) < (size_t)n) ++idbits;
  int split = shift + idbits > 32 ? shift + idbits - 32 : 0;
  while (split < shift && (double)n / (double)(rows << split) > 64.0) ++split;
  return split > shift ? shift : split;
}

size_t cell_sort_scratch_bytes(int n, size_t rows, int shift) {
  const size_t segs = rows << cell_sort_split(n, rows, shift);
  const size_t nb = (segs + SCAN_TILE - 1) / SCAN_TILE;
  // counts, cursors, segment starts, scan partials, buckets, radix scratch (hi, lo)
  return (3 * segs + 1 + nb + 64 + 3 * (size_t)n) * sizeof(uint32_t) + 4 * 256;
}

void launch_cell_sort(const uint32_t* keys, const uint32_t* order, int n, int shift,
                      size_t rows, uint32_t* keys_sorted, uint32_t* ids_sorted,
                      uint32_t* row_start, void* scratch, const Vec3* pay_in, Vec3* pay_out,
                      uint32_t* inv, hipStream_t s) {
  const int split = cell_sort_split(n, rows, shift);
  const int sshift = shift - split;  // key >> sshift = segment
  const size_t segs = rows << split;
  const size_t nb = (segs + SCAN_TILE - 1) / SCAN_TILE;
  uint32_t* cnt = (uint32_t*)scratch;
  uint32_t* cursor = cnt + segs;
  uint32_t* seg_start = cursor + segs;
  uint32_t* partial = seg_start + segs + 1;
  uint32_t* bucket = partial + nb + 64;
  uint32_t* tmp_hi = bucket + n;
  uint32_t* tmp_lo = tmp_hi + n;
  // (segment << 6 | lane) fits 32 bits below the end marker ~0 for the wavefront sort of
  // the segment numbers
  const bool packed = segs <= ((size_t)1 << 25);
  fill_u32_kernel<<<grid_for(segs, TB * 8) < 1024 ? grid_for(segs, TB * 8) : 1024, TB, 0, s>>>(
      cnt, segs, 0u);
  if (packed)
    row_count_kernel<<<grid_for(n, TB * GROUPS), TB, 0, s>>>(keys, order, n, sshift, cnt);
  else
    row_count_loop_kernel<<<grid_for(n, TB), TB, 0, s>>>(keys, order, n, sshift, cnt);
  scan_reduce_kernel<<<(int)nb, TB, 0, s>>>(cnt, segs, partial);
  scan_partials_kernel<<<1, TB, 0, s>>>(partial, (int)nb);
  scan_write_kernel<<<(int)nb, TB, 0, s>>>(cnt, segs, partial, (uint32_t)n, row_start, cursor,
                                            seg_start, split);
  if (packed)
    bucket_kernel<<<grid_for(n, TB * GROUPS), TB, 0, s>>>(keys, order, n, sshift, cursor, bucket);
  else
    bucket_loop_kernel<<<grid_for(n, TB), TB, 0, s>>>(keys, order, n, sshift, cursor, bucket);
  RowSortArgs a{};
  a.keys = keys;
  a.row_start = seg_start;
  a.bucket = bucket;
  a.keys_sorted = keys_sorted;
  a.ids_sorted = ids_sorted;
  a.pay_in = pay_in;
  a.pay_out = pay_out;
  a.inv = inv;
  a.tmp_hi = tmp_hi;
  a.tmp_lo = tmp_lo;
  a.shift = sshift;
  a.zmask = (1u << sshift) - 1u;
  a.idbits = 0;
  while (a.idbits < 32 && ((size_t)1 << a.idbits) < (size_t)n) ++a.idbits;
  a.rows = segs;
  // one wavefront per WAVE_ROWS segments (the grid is not capped at the resident count: waiting
  // workgroups start as others finish)
  const size_t need = (segs + WAVE_ROWS * (TB / 64) - 1) / (WAVE_ROWS * (TB / 64));
  const bool narrow = sshift + a.idbits <= 32;
  if (narrow)
    row_sort_wave_kernel<uint32_t><<<(int)need, TB, 0, s>>>(a);
  else
    row_sort_wave_kernel<uint64_t><<<(int)need, TB, 0, s>>>(a);
  const int blk = narrow ? resident_grid<row_sort_block_kernel<uint32_t>, TB>()
                         : resident_grid<row_sort_block_kernel<uint64_t>, TB>();
  // rows tested per workgroup step: TB, halved (down to 32) while that leaves resident
  // workgroups without rows
  a.block_rows = TB;
  while (a.block_rows > 32 && segs / (size_t)a.block_rows < (size_t)blk) a.block_rows /= 2;
  const size_t chunks = (segs + a.block_rows - 1) / a.block_rows;
  const int grid = chunks < (size_t)blk ? (int)chunks : blk;
  if (narrow)
    row_sort_block_kernel<uint32_t><<<grid, TB, 0, s>>>(a);
  else
    row_sort_block_kernel<uint64_t><<<grid, TB, 0, s>>>(a);
}

}  // namespace pmr
