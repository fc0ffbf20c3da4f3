// CIC paint building blocks shared by the paint kernels (cic.hip) and the paint fused with
// the first FFT pass (fft_kernels.h): sorted-stream chunks, the wave-level segmented scan and
// the phase-ordered deposit into a wavefront's LDS rows. Include inside namespace pmr's
// anonymous namespace.
#pragma once


// Segmented inclusive scan over the 64 lanes by equal key, on DPP lane moves (VALU, no
// LDS): row_shr 1, 2, 4, 8 inside each row of 16 lanes, then row_bcast 15 and row_bcast 31
// across rows. Keys are sorted across the lanes, so "source key == my key" means the
// source lane is in my segment. A key whose DPP source is out of range or in a row the
// move leaves out reads ~0 (at most the key of the very last cell, whose added value is
// then 0); the in-row shifts read values with the bound control (out of range reads 0)
// and no old operand, so no register has to be cleared before them, and the row
// broadcasts, which leave rows out, read 0 there from a cleared old operand. The
// neighbour keys (previous and next lane across the whole wavefront) come from the DPP
// wavefront shifts, VALU moves with no LDS round trip; lanes 0 and 63, which have no
// neighbour there, are handled by the lane tests that follow.
template <int CTRL, int RMASK>
__device__ __forceinline__ float dpp_f(float src) {
  if constexpr (RMASK == 0xF)  // every row written: out-of-range lanes read 0
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(src), CTRL, RMASK, 0xF, true));
  else  // rows left out keep the old operand: 0
    return __int_as_float(
        __builtin_amdgcn_update_dpp(0, __float_as_int(src), CTRL, RMASK, 0xF, false));
}
template <int CTRL, int RMASK>
__device__ __forceinline__ uint32_t dpp_k(uint32_t src) {
  return (uint32_t)__builtin_amdgcn_update_dpp(-1, (int)src, CTRL, RMASK, 0xF, false);
}

template <int NV, int CTRL, int RMASK>
__device__ __forceinline__ void seg_step(float (&v)[NV], uint32_t key) {
  const uint32_t ks = dpp_k<CTRL, RMASK>(key);
  float t[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) t[q] = dpp_f<CTRL, RMASK>(v[q]);
  if (ks == key) {
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] += t[q];
  }
}

// Only the steps the chunk needs run (wave-uniform): with eq = lanes whose key equals the
// previous lane's, the longest run of set bits bounds the within-row shifts, and the
// row-crossing steps run only when a segment crosses lane 16/48 or 32.
template <int NV>
__device__ __forceinline__ void seg_scan(float (&v)[NV], uint32_t key) {
  // wave_shr:1
  const uint32_t kp = (uint32_t)__builtin_amdgcn_mov_dpp((int)key, 0x138, 0xF, 0xF, true);
  const int lane = threadIdx.x & 63;
  const uint64_t eq = __ballot(lane > 0 && kp == key);
  if (eq == 0) return;
  int run = 0;  // longest run of ones in eq
  for (uint64_t m = eq; m; m &= (m >> 1)) ++run;
  seg_step<NV, 0x111, 0xF>(v, key);                       // row_shr:1
  if (run >= 2) seg_step<NV, 0x112, 0xF>(v, key);         // row_shr:2
  if (run >= 4) seg_step<NV, 0x114, 0xF>(v, key);         // row_shr:4
  if (run >= 8) seg_step<NV, 0x118, 0xF>(v, key);         // row_shr:8
  if (eq & ((1ull << 16) | (1ull << 48))) seg_step<NV, 0x142, 0xA>(v, key);  // row_bcast:15
  if (eq & (1ull << 32)) seg_step<NV, 0x143, 0xC>(v, key);  // row_bcast:31
}

// One 64-particle chunk of a source run: per lane the four (oy, oz) weights of each channel.
template <int C>
struct Chunk {
  uint32_t key;
  int sy, iz;
  bool ok;
  float v[4 * C];
};

template <int C>
__device__ __forceinline__ void load_chunk(const PaintArgs& a, uint32_t j, uint32_t end, int ox,
                                           Chunk<C>& ch) {
  const int lane = threadIdx.x & 63;
  const int nm = a.nm;
  ch.ok = j < end;
  ch.key = 0xffffffffu - lane;  // never equal across lanes when invalid
  ch.sy = 0;
  ch.iz = 0;
#pragma unroll
  for (int q = 0; q < 4 * C; ++q) ch.v[q] = 0.f;
  if (ch.ok) {
    const uint32_t key = a.keys[j];
    const Vec3 f = a.frac[j];
    ch.key = key;
    ch.iz = (int)(key & (uint32_t)(nm - 1));
    ch.sy = (int)((key >> a.log_nm) & (uint32_t)(nm - 1));
    const float wx = ox ? f.x : 1.f - f.x;
    float val[C];
    if constexpr (C == 1) {
      val[0] = a.mass * wx;
    } else {
      const Vec3 u = a.val[j];
      val[0] = u.x * wx;
      val[1] = u.y * wx;
      val[2] = u.z * wx;
    }
    const float wy0 = 1.f - f.y, wy1 = f.y, wz0 = 1.f - f.z, wz1 = f.z;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      ch.v[4 * c + 0] = val[c] * wy0 * wz0;
      ch.v[4 * c + 1] = val[c] * wy0 * wz1;
      ch.v[4 * c + 2] = val[c] * wy1 * wz0;
      ch.v[4 * c + 3] = val[c] * wy1 * wz1;
    }
  }
}

// Last lane of each run adds the run's sums to its two target rows. The accumulator is
// private to the wavefront and, within one phase below, the tails of a chunk touch
// distinct words, so a plain read-add-write is race-free inside a phase. Different phases
// (and chunks) may touch the same word from different lanes: a compiler barrier keeps the
// phases in program order, and LDS instructions of one wavefront execute in issue order,
// so every word receives its additions in one fixed order.
#define PMR_PHASE_FENCE() asm volatile("" ::: "memory")

// Float slot of cell iz in an LDS row: plain (iz), or, for rows that the z-pass FFT then
// transforms in place, the padded complex layout (one spare complex slot every 32 complex
// values: real point iz is half of complex point iz / 2).
template <bool PAD>
__device__ __forceinline__ int row_slot(int iz) {
  if constexpr (PAD) {
    const int k = iz >> 1;
    return 2 * (k + (k >> 5)) + (iz & 1);
  }
  return iz;
}

// acc rows: [TY][C] rows of rp floats each.
template <int C, int TY, bool PAD = false>
__device__ __forceinline__ void deposit(const Chunk<C>& ch, float* acc, int nm, int iy0, int rp) {
  const int lane = threadIdx.x & 63;
  // wave_shl:1
  const uint32_t kn = (uint32_t)__builtin_amdgcn_mov_dpp((int)ch.key, 0x130, 0xF, 0xF, true);
  const int ok_next = __builtin_amdgcn_mov_dpp((int)ch.ok, 0x130, 0xF, 0xF, true);
  const bool tail = ch.ok && (lane == 63 || !ok_next || kn != ch.key);
  const int iz1 = (ch.iz + 1) & (nm - 1);
#pragma unroll
  for (int ph = 0; ph < 4; ++ph) {
    const int oy = ph >> 1, oz = ph & 1;
    const int jt = ((ch.sy + oy) & (nm - 1)) - iy0;
    PMR_PHASE_FENCE();
    if (tail && jt >= 0 && jt < TY) {
      float* row = acc + (size_t)jt * C * rp + row_slot<PAD>(oz ? iz1 : ch.iz);
#pragma unroll
      for (int c = 0; c < C; ++c) row[c * rp] = row[c * rp] + ch.v[4 * c + 2 * oy + oz];
    }
    PMR_PHASE_FENCE();
  }
}

// One target row per wavefront (TY = 1): a particle of source row sy reaches that row
// through one corner row only (oy = 1 from row iy0 - 1, oy = 0 from row iy0; its other
// corner row belongs to another wavefront), so a chunk carries the 2 C values of that oy:
// half the weights and half the scan of the general chunk. The same lanes deposit the same
// values in the same phases as the general path, so the rows are bitwise the same.
template <int C>
struct Chunk1 {
  uint32_t key;
  int iz, oy;
  bool ok;
  float v[2 * C];
};

template <int C>
__device__ __forceinline__ void load_chunk1(const PaintArgs& a, uint32_t j, uint32_t end, int ox,
                                            int iy0, Chunk1<C>& ch) {
  const int lane = threadIdx.x & 63;
  const int nm = a.nm;
  ch.ok = j < end;
  ch.key = 0xffffffffu - lane;  // never equal across lanes when invalid
  ch.iz = 0;
  ch.oy = 0;
#pragma unroll
  for (int q = 0; q < 2 * C; ++q) ch.v[q] = 0.f;
  if (ch.ok) {
    const uint32_t key = a.keys[j];
    const Vec3 f = a.frac[j];
    ch.key = key;
    ch.iz = (int)(key & (uint32_t)(nm - 1));
    const int sy = (int)((key >> a.log_nm) & (uint32_t)(nm - 1));
    ch.oy = sy == iy0 ? 0 : 1;
    const float wx = ox ? f.x : 1.f - f.x;
    float val[C];
    if constexpr (C == 1) {
      val[0] = a.mass * wx;
    } else {
      const Vec3 u = a.val[j];
      val[0] = u.x * wx;
      val[1] = u.y * wx;
      val[2] = u.z * wx;
    }
    const float wy = ch.oy ? f.y : 1.f - f.y, wz0 = 1.f - f.z, wz1 = f.z;
#pragma unroll
    for (int c = 0; c < C; ++c) {
      ch.v[2 * c + 0] = val[c] * wy * wz0;
      ch.v[2 * c + 1] = val[c] * wy * wz1;
    }
  }
}

template <int C, bool PAD = false>
__device__ __forceinline__ void deposit1(const Chunk1<C>& ch, float* acc, int nm, int rp) {
  const int lane = threadIdx.x & 63;
  // wave_shl:1
  const uint32_t kn = (uint32_t)__builtin_amdgcn_mov_dpp((int)ch.key, 0x130, 0xF, 0xF, true);
  const int ok_next = __builtin_amdgcn_mov_dpp((int)ch.ok, 0x130, 0xF, 0xF, true);
  const bool tail = ch.ok && (lane == 63 || !ok_next || kn != ch.key);
  const int iz1 = (ch.iz + 1) & (nm - 1);
#pragma unroll
  for (int ph = 0; ph < 4; ++ph) {
    const int oy = ph >> 1, oz = ph & 1;
    PMR_PHASE_FENCE();
    if (tail && ch.oy == oy) {
      float* row = acc + row_slot<PAD>(oz ? iz1 : ch.iz);
#pragma unroll
      for (int c = 0; c < C; ++c) row[c * rp] = row[c * rp] + ch.v[2 * c + oz];
    }
    PMR_PHASE_FENCE();
  }
}

// Chunks of 64 particles loaded together before their scans and deposits (memory-level
// parallelism of a wave's walk over its source rows). One at a time measured 1-3% faster
// for the paints than two (fewer live registers; the loads of other resident waves cover
// the latency) and four 6-20% slower.
#ifndef PMR_PAINT_CHUNKS
#define PMR_PAINT_CHUNKS 1
#endif

// Deposits of all particles that reach the TY target rows [iy0, iy0 + TY) of plane ix of one
// item, into the wavefront's rows acc (zeroed by the caller): the two source planes ix - 1
// and ix, each as one or two contiguous runs of source rows. Chunks are deposited in stream
// order, so the result does not depend on how many are in flight.
template <int C, int TY, bool PAD = false>
__device__ __forceinline__ void paint_rows(const PaintArgs& a, int item, int ix, int iy0,
                                           float* acc, int rp) {
  constexpr int CH = PMR_PAINT_CHUNKS;
  const int lane = threadIdx.x & 63;
  const int nm = a.nm;
  const int rows_item = item * nm * nm;
  // main runs of source rows [iy0 - 1, iy0 + TY - 1] of both planes (from row 0 when iy0 - 1
  // wraps; row nm - 1 is then a second run)
  const int lo0 = iy0 == 0 ? 0 : iy0 - 1, hi0 = iy0 + TY - 1;
  uint32_t beg0[2], end0[2];
#pragma unroll
  for (int ox = 0; ox < 2; ++ox) {
    const int rbase = rows_item + ((ix - ox + nm) & (nm - 1)) * nm;
    beg0[ox] = a.row_start[rbase + lo0];
    end0[ox] = a.row_start[rbase + hi0 + 1];
  }
#pragma unroll 1
  for (int ox = 0; ox < 2; ++ox) {
    const int rbase = rows_item + ((ix - ox + nm) & (nm - 1)) * nm;
#pragma unroll 1
    for (int run = 0; run < 2; ++run) {
      uint32_t beg, end;
      if (run == 0) {
        beg = ox == 0 ? beg0[0] : beg0[1];
        end = ox == 0 ? end0[0] : end0[1];
      } else {
        if (iy0 != 0) continue;
        beg = a.row_start[rbase + nm - 1];
        end = a.row_start[rbase + nm];
      }
#pragma unroll 1
      for (uint32_t c0 = beg; c0 < end; c0 += 64 * CH) {
        if constexpr (TY == 1) {
          Chunk1<C> ch[CH];
#pragma unroll
          for (int q = 0; q < CH; ++q)
            load_chunk1<C>(a, c0 + 64 * q + lane, end, ox, iy0, ch[q]);
#pragma unroll
          for (int q = 0; q < CH; ++q) seg_scan<2 * C>(ch[q].v, ch[q].key);
#pragma unroll
          for (int q = 0; q < CH; ++q)
            if (q == 0 || c0 + 64 * q < end) deposit1<C, PAD>(ch[q], acc, nm, rp);
        } else {
          Chunk<C> ch[CH];
#pragma unroll
          for (int q = 0; q < CH; ++q) load_chunk<C>(a, c0 + 64 * q + lane, end, ox, ch[q]);
#pragma unroll
          for (int q = 0; q < CH; ++q) seg_scan<4 * C>(ch[q].v, ch[q].key);
#pragma unroll
          for (int q = 0; q < CH; ++q)
            if (q == 0 || c0 + 64 * q < end) deposit<C, TY, PAD>(ch[q], acc, nm, iy0, rp);
        }
      }
    }
  }
}
