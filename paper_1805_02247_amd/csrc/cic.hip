// Particles: cell keys, the stable (cell, id) sort, cloud-in-cell paint and readout,
// kick/drift and their adjoints.
//
// Particle state is kept in Lagrangian (id) order: id = (i*Np + j)*Np + k for the lattice
// site (i, j, k), which keeps neighbouring ids close in space through the evolution, so
// the per-particle gathers below stay cache friendly without moving the state.
// Positions are FP64 [B][3][Np^3]; momenta and adjoints FP32 [B][3][Np^3].
//
// Keys carry the batch item: key = item*Nm^3 + (ix*Nm + iy)*Nm + iz, with (ix, iy, iz)
// the lower CIC corner computed in FP64. A stable LSD radix sort of (key, id) gives the
// unique (key, id) order; rows (item, ix, iy) are then contiguous and `row_start` indexes
// them.
//
// Paint is owner-computes and atomic-free across the device: one wavefront owns TY
// consecutive target rows of Nm cells in LDS and walks the source rows that can reach them
// (paint_kernels.h). Inside a source row the particles arrive sorted by iz, so a segmented
// scan over the 64 lanes sums equal-cell runs and only the last lane of each run touches
// LDS: each LDS word is written by one lane per instruction, in program order, so the
// result is bitwise reproducible.
//
// The forward readout (kick_drift_kernel) gathers in id order; the step adjoint gathers its
// two position terms in sort order (adjoint_positions_kernel: neighbouring lanes read
// neighbouring cells, as in the paint) and applies the kick and drift transposes in id
// order (adjoint_update_kernel).
#include "pmr_internal.h"

namespace pmr {
namespace {

constexpr int TB = 256;  // threads per block for per-particle kernels

// ---------------------------------------------------------------- keys
// Key and CIC fractions (id order) of one particle on an nm mesh.
__device__ __forceinline__ uint32_t key_frac(const double* xyz, double scale, int nm, uint32_t item,
                                             Vec3* frac) {
  double f[3];
  const int ix = cic_corner(xyz[0], scale, nm, &f[0]);
  const int iy = cic_corner(xyz[1], scale, nm, &f[1]);
  const int iz = cic_corner(xyz[2], scale, nm, &f[2]);
  *frac = Vec3{(float)f[0], (float)f[1], (float)f[2]};
  const uint32_t cells = (uint32_t)nm * nm * nm;
  return item * cells + ((uint32_t)ix * nm + iy) * nm + iz;
}

__global__ void keys_kernel(const double* __restrict__ x, int log_np3, int total, double scale,
                            int nm, uint32_t* __restrict__ keys, Vec3* __restrict__ frac) {
  const int g = blockIdx.x * TB + threadIdx.x;
  if (g >= total) return;
  const size_t np3 = (size_t)1 << log_np3;
  const uint32_t item = g >> log_np3;
  const size_t id = g & (np3 - 1);
  const double* xi = x + (size_t)item * 3 * np3 + id;
  double p[3] = {xi[0], xi[np3], xi[2 * np3]};
  Vec3 f;
  keys[g] = key_frac(p, scale, nm, item, &f);
  if (frac) frac[g] = f;
}

// ---------------------------------------------------------------- radix sort
#ifndef PMR_SORT_WAVES
#define PMR_SORT_WAVES 8
#endif
constexpr int SORT_TILE = 4096;  // keys per tile
constexpr int SORT_WAVES = PMR_SORT_WAVES;
constexpr int SORT_TB = SORT_WAVES * PMR_WAVE;
constexpr int SORT_ITEMS = SORT_TILE / SORT_TB;

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int l = threadIdx.x & 63;
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// Lanes of this wavefront (among `valid`) whose digit equals mine.
template <int D>
__device__ __forceinline__ uint64_t match_digit(uint32_t d, uint64_t valid) {
  uint64_t m = valid;
#pragma unroll
  for (int b = 0; b < D; ++b) {
    const bool bit = (d >> b) & 1u;
    const uint64_t bal = __ballot(bit);
    m &= bit ? bal : ~bal;
  }
  return m;
}

// Digit histogram of each tile: hist[digit * nblocks + block].
template <int D>
__global__ __launch_bounds__(TB) void radix_hist_kernel(const uint32_t* __restrict__ keys, int n,
                                                        int shift, uint32_t* __restrict__ hist) {
  constexpr int NBK = 1 << D;
  __shared__ uint32_t cnt[NBK];
  for (int i = threadIdx.x; i < NBK; i += TB) cnt[i] = 0;
  __syncthreads();
  const size_t base = (size_t)blockIdx.x * SORT_TILE;
  for (int i = threadIdx.x; i < SORT_TILE; i += TB) {
    const size_t j = base + i;
    if (j < (size_t)n) atomicAdd(&cnt[(keys[j] >> shift) & (NBK - 1)], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < NBK; i += TB) hist[(size_t)i * gridDim.x + blockIdx.x] = cnt[i];
}

// Stable scatter. Key j of the tile is handled by wave w = (j / 64) / ITEMS in order, so
// ranks follow j: local rank = (same digit in earlier waves) + (same digit earlier in this
// wave). The tile is first placed in LDS in digit order, then each digit's run is written
// to its global range [offset[digit][block], ...) contiguously.
// ids_in == nullptr means identity payload (id = index).
template <int D>
__global__ __launch_bounds__(SORT_TB) void radix_scatter_kernel(const uint32_t* __restrict__ keys_in,
                                                           const uint32_t* __restrict__ ids_in,
                                                           int n, int shift,
                                                           const uint32_t* __restrict__ offsets,
                                                           const uint32_t* __restrict__ digit_total,
                                                           uint32_t* __restrict__ keys_out,
                                                           uint32_t* __restrict__ ids_out,
                                                           const Vec3* __restrict__ pay_in,
                                                           Vec3* __restrict__ pay_out,
                                                           uint32_t* __restrict__ inv_out) {
  constexpr int NBK = 1 << D;
  __shared__ uint32_t cnt[SORT_WAVES][NBK];
  __shared__ uint32_t dstart[NBK];   // block-local start of each digit
  __shared__ uint32_t gbase[NBK];    // global start of each digit for this block
  __shared__ uint32_t skey[SORT_TILE];
  __shared__ uint32_t sid[SORT_TILE];
  __shared__ uint32_t wsum[2 * SORT_WAVES];
  const int w = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  for (int i = threadIdx.x; i < SORT_WAVES * NBK; i += SORT_TB) (&cnt[0][0])[i] = 0;
  __syncthreads();
  // consecutive tiles on one XCD: their runs of each digit are adjacent in the output, so
  // the partial lines they write meet in one L2
  const int tile = xcd_block(blockIdx.x, gridDim.x);
  const size_t tile0 = (size_t)tile * SORT_TILE;
  const size_t base = tile0 + (size_t)w * PMR_WAVE * SORT_ITEMS;
  uint32_t key[SORT_ITEMS], id[SORT_ITEMS], rank[SORT_ITEMS];
  const uint64_t lt = lanemask_lt();
#pragma unroll
  for (int it = 0; it < SORT_ITEMS; ++it) {
    const size_t j = base + (size_t)it * PMR_WAVE + lane;
    const bool ok = j < (size_t)n;
    key[it] = ok ? keys_in[j] : 0u;
    id[it] = ok ? (ids_in ? ids_in[j] : (uint32_t)j) : 0u;
    const uint32_t d = (key[it] >> shift) & (NBK - 1);
    const uint64_t valid = __ballot(ok);
    const uint64_t m = match_digit<D>(d, valid);
    uint32_t r = 0;
    if (ok) r = cnt[w][d] + (uint32_t)__popcll(m & lt);
    rank[it] = r;
    // the lowest lane of each digit group advances the running count
    if (ok && (m & lt) == 0) cnt[w][d] += (uint32_t)__popcll(m);
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0): LDS update visible to the next item
  }
  __syncthreads();
  // per digit: exclusive prefix over waves, and the block total
  constexpr int Q = (NBK + SORT_TB - 1) / SORT_TB;
  uint32_t tot_local[Q], dig_tot[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int d = threadIdx.x + q * SORT_TB;
    uint32_t run = 0, dt = 0;
    if (d < NBK) {
#pragma unroll
      for (int ww = 0; ww < SORT_WAVES; ++ww) {
        const uint32_t c = cnt[ww][d];
        cnt[ww][d] = run;
        run += c;
      }
      gbase[d] = offsets[(size_t)d * gridDim.x + tile];
      dt = digit_total[d];
    }
    tot_local[q] = run;
    dig_tot[q] = dt;
  }
  // exclusive scans over digits (digit d = thread + q * SORT_TB) of the block totals (start
  // of each digit in the tile) and of the global digit totals (start of each digit's range)
  {
    uint32_t carry = 0, gcarry = 0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const uint32_t v = tot_local[q], gv = dig_tot[q];
      // wave-level inclusive scans
      uint32_t x = v, gx = gv;
#pragma unroll
      for (int dd = 1; dd < 64; dd <<= 1) {
        const uint32_t y = __shfl_up(x, dd, 64);
        const uint32_t gy = __shfl_up(gx, dd, 64);
        if (lane >= dd) {
          x += y;
          gx += gy;
        }
      }
      if (lane == 63) {
        wsum[w] = x;
        wsum[SORT_WAVES + w] = gx;
      }
      __syncthreads();
      uint32_t wpre = 0, total = 0, gpre = 0, gtotal = 0;
#pragma unroll
      for (int ww = 0; ww < SORT_WAVES; ++ww) {
        const uint32_t sv = wsum[ww], gs = wsum[SORT_WAVES + ww];
        if (ww < w) {
          wpre += sv;
          gpre += gs;
        }
        total += sv;
        gtotal += gs;
      }
      const int d = threadIdx.x + q * SORT_TB;
      if (d < NBK) {
        dstart[d] = carry + wpre + x - v;
        gbase[d] += gcarry + gpre + gx - gv;
      }
      carry += total;
      gcarry += gtotal;
      __syncthreads();
    }
  }
  __syncthreads();
  // place the tile in LDS in (digit, rank) order
#pragma unroll
  for (int it = 0; it < SORT_ITEMS; ++it) {
    const size_t j = base + (size_t)it * PMR_WAVE + lane;
    if (j < (size_t)n) {
      const uint32_t d = (key[it] >> shift) & (NBK - 1);
      const uint32_t lp = dstart[d] + cnt[w][d] + rank[it];
      skey[lp] = key[it];
      sid[lp] = id[it];
    }
  }
  __syncthreads();
  const int count = (int)min((size_t)SORT_TILE, (size_t)n - tile0);
  for (int e = threadIdx.x; e < count; e += SORT_TB) {
    const uint32_t k = skey[e];
    const uint32_t d = (k >> shift) & (NBK - 1);
    const uint32_t dst = gbase[d] + (uint32_t)e - dstart[d];
    const uint32_t idv = sid[e];
    keys_out[dst] = k;
    ids_out[dst] = idv;
    if (pay_out) pay_out[dst] = pay_in[idv];
    if (inv_out) inv_out[idv] = dst;
  }
}

// ---------------------------------------------------------------- exclusive scan (u32)
constexpr int SCAN_ITEMS = 16;
constexpr int SCAN_TILE = TB * SCAN_ITEMS;

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* sh, uint32_t* total) {
  // sh: TB words
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int d = 1; d < TB; d <<= 1) {
    uint32_t a = t >= d ? sh[t - d] : 0u;
    __syncthreads();
    sh[t] += a;
    __syncthreads();
  }
  const uint32_t incl = sh[t];
  *total = sh[TB - 1];
  __syncthreads();
  return incl - v;
}

// Per digit (one block each): exclusive scan of the tile histograms over tiles, giving each
// tile's start within the digit's range, and the digit's total.
__global__ __launch_bounds__(TB) void digit_scan_kernel(const uint32_t* __restrict__ hist, int nb,
                                                        uint32_t* __restrict__ offs,
                                                        uint32_t* __restrict__ digit_total) {
  __shared__ uint32_t sh[TB];
  const size_t row = (size_t)blockIdx.x * nb;
  uint32_t carry = 0;
  for (int b0 = 0; b0 < nb; b0 += SCAN_TILE) {
    const int t0 = b0 + threadIdx.x * SCAN_ITEMS;
    uint32_t v[SCAN_ITEMS];
    uint32_t sum = 0;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
      v[i] = t0 + i < nb ? hist[row + t0 + i] : 0u;
      sum += v[i];
    }
    uint32_t tot;
    uint32_t run = carry + block_exclusive_scan(sum, sh, &tot);
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
      if (t0 + i < nb) offs[row + t0 + i] = run;
      run += v[i];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) digit_total[blockIdx.x] = carry;
}

// ---------------------------------------------------------------- row starts
// row_start[r] = first sorted position whose row (key >> log_nm) is >= r; r = 0..rows.
__global__ void row_start_kernel(const uint32_t* __restrict__ keys, int n, int log_nm, int rows,
                                 uint32_t* __restrict__ row_start) {
  const int j = blockIdx.x * TB + threadIdx.x;
  if (j > n) return;
  const int r_hi = j < n ? (int)(keys[j] >> log_nm) : rows;
  const int r_lo = j > 0 ? (int)(keys[j - 1] >> log_nm) : -1;
  for (int r = r_lo + 1; r <= r_hi; ++r) row_start[r] = j;
}

// ---------------------------------------------------------------- sorted particle streams
// Per sorted position j: the CIC fractions of particle ids[j] (FP64 rule, rounded to FP32).
__global__ __launch_bounds__(TB) void stream_frac_kernel(const uint32_t* __restrict__ ids,
                                                         const double* __restrict__ x, int total,
                                                         int log_np3, double scale, int nm,
                                                         Vec3* __restrict__ frac) {
  const int j = blockIdx.x * TB + threadIdx.x;
  if (j >= total) return;
  const size_t np3 = (size_t)1 << log_np3;
  const uint32_t g = ids[j];
  const size_t pi = (size_t)(g >> log_np3) * 3 * np3 + (g & (np3 - 1));
  double fx, fy, fz;
  cic_corner(x[pi], scale, nm, &fx);
  cic_corner(x[pi + np3], scale, nm, &fy);
  cic_corner(x[pi + 2 * np3], scale, nm, &fz);
  frac[j] = Vec3{(float)fx, (float)fy, (float)fz};
}

// Per sorted position j: the payload of particle ids[j] (id-order Vec3 -> sorted order).
__global__ __launch_bounds__(TB) void stream_gather_kernel(const uint32_t* __restrict__ ids,
                                                           const Vec3* __restrict__ src,
                                                           int total, Vec3* __restrict__ dst) {
  const int j = xcd_block(blockIdx.x, gridDim.x) * TB + threadIdx.x;
  if (j >= total) return;
  dst[j] = src[ids[j]];
}

// ---------------------------------------------------------------- paint
// One wavefront owns TY consecutive target rows (item, ix, iy0 .. iy0+TY-1), accumulated
// in LDS. For each ox in {0, 1} its source rows (ix - ox, iy0 - 1 .. iy0 + TY - 1) are one
// contiguous run of the sorted stream (two runs when iy0 - 1 wraps), walked in full 64-lane
// chunks. A particle in source row sy reaches target rows sy and sy + 1. Within a chunk the
// keys are sorted, so a segmented scan sums equal-(sy, iz) runs and only the last lane of a
// run writes, to a cell no other lane of that instruction touches: every LDS word receives
// its additions in one fixed order and the mesh is bitwise reproducible.
#include "paint_kernels.h"

template <int C, int TY>
__global__ __launch_bounds__(TB) void paint_kernel(PaintArgs a) {
  extern __shared__ float acc_all[];
  const int w = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int nm = a.nm;
  const int seg = xcd_block(blockIdx.x, gridDim.x) * (TB / 64) + w;  // (item, ix, segment)
  const int segs_per_x = nm / TY;
  const int item = seg / (nm * segs_per_x);
  const int rr = seg - item * nm * segs_per_x;
  const int ix = rr / segs_per_x;
  const int iy0 = (rr - ix * segs_per_x) * TY;
  float* acc = acc_all + (size_t)w * TY * C * nm;  // [TY][C][nm]
  for (int i = lane; i < TY * C * nm; i += 64) acc[i] = 0.f;
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_s_waitcnt(0xc07f);
  paint_rows<C, TY>(a, item, ix, iy0, acc, nm);
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_s_waitcnt(0xc07f);
  const size_t cells = (size_t)nm * nm * nm;
  for (int t = 0; t < TY; ++t) {
    float* dst = a.out + (size_t)item * C * cells + ((size_t)ix * nm + iy0 + t) * nm;
    for (int c = 0; c < C; ++c)
      for (int i = lane; i < nm; i += 64) dst[c * cells + i] = acc[(t * C + c) * nm + i] - a.bias;
  }
}

// ---------------------------------------------------------------- gathers
struct Corner {
  int i0[3], i1[3];
  float f[3];
};

__device__ __forceinline__ Corner corner_of(const double* xyz, double scale, int nm) {
  Corner c;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double f;
    c.i0[a] = cic_corner(xyz[a], scale, nm, &f);
    c.i1[a] = (c.i0[a] + 1) & (nm - 1);
    c.f[a] = (float)f;
  }
  return c;
}

// Cell index within one item's mesh (nm^3 <= 2^27 fits 32 bits).
__device__ __forceinline__ uint32_t cidx(const Corner& c, int ox, int oy, int oz, int nm) {
  const uint32_t ix = ox ? c.i1[0] : c.i0[0];
  const uint32_t iy = oy ? c.i1[1] : c.i0[1];
  const uint32_t iz = oz ? c.i1[2] : c.i0[2];
  return (ix * (uint32_t)nm + iy) * (uint32_t)nm + iz;
}

struct StepArgs {
  const double* x;    // [B][3][Np^3] positions x_i
  double* x_next;     // positions x_{i+1}
  float* p;           // momenta, updated in place
  const Vec3* F;    // [B][nm^3] interleaved force mesh (Fx, Fy, Fz) at x_i
  uint32_t* keys;     // keys of x_{i+1} (nullable)
  Vec3* frac;       // CIC fractions of x_{i+1} on the key mesh, id order
  int log_np3, nm, total;
  double scale, box;
  float kick;
  double drift;
  int key_nm;         // mesh of the keys emitted for x_{i+1}
  double key_scale;
};

// p += kick * F(x_i);  x_{i+1} = wrap(x_i + drift * p);  key(x_{i+1})
__global__ __launch_bounds__(TB) void kick_drift_kernel(StepArgs a) {
  const int g = xcd_block(blockIdx.x, gridDim.x) * TB + threadIdx.x;
  if (g >= a.total) return;
  const size_t np3 = (size_t)1 << a.log_np3;
  const int item = g >> a.log_np3;
  const size_t id = g & (np3 - 1);
  const size_t pi = (size_t)item * 3 * np3 + id;
  double xyz[3] = {a.x[pi], a.x[pi + np3], a.x[pi + 2 * np3]};
  const int nm = a.nm;
  const Corner c = corner_of(xyz, a.scale, nm);
  const size_t cells = (size_t)nm * nm * nm;
  const Vec3* F = a.F + (size_t)item * cells;
  float fa[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int o = 0; o < 8; ++o) {
    const int ox = o >> 2, oy = (o >> 1) & 1, oz = o & 1;
    const float w = (ox ? c.f[0] : 1.f - c.f[0]) * (oy ? c.f[1] : 1.f - c.f[1]) *
                     (oz ? c.f[2] : 1.f - c.f[2]);
    const Vec3 f = F[cidx(c, ox, oy, oz, nm)];
    fa[0] += w * f.x;
    fa[1] += w * f.y;
    fa[2] += w * f.z;
  }
  double xn[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const float pq = a.p[pi + q * np3] + a.kick * fa[q];
    a.p[pi + q * np3] = pq;
    xn[q] = wrap_box(xyz[q] + a.drift * (double)pq, a.box);
    a.x_next[pi + q * np3] = xn[q];
  }
  if (a.keys) {
    Vec3 f;
    a.keys[g] = key_frac(xn, a.key_scale, a.key_nm, item, &f);
    a.frac[g] = f;
  }
}

// Position gradient of the step adjoint, in sort order (the transpose of the paint, so the
// mesh reads are as coherent as the paint's writes):
//   g(p) = sum_cell dW(x_p - cell)/dx * (sum_a Fbar_a(p) F_a(cell) + mass * dbar(cell))
// with the corner cell and fractions of particle p taken from its key and sorted fractions
// (the same FP64-derived values the paint used) and Fbar(p) from the sorted adjoint-paint
// stream. Written to g_out[id] (id order) for the update below.
struct AdjPosArgs {
  const uint32_t* keys;  // sorted keys
  const Vec3* frac;    // sorted fractions
  const Vec3* fbar;    // sorted Fbar (nullable: final-paint adjoint, no force term)
  const uint32_t* ids;   // sorted ids
  const Vec3* F;       // interleaved force mesh at x_i [B][nm^3] (nullable with fbar)
  const float* dbar;     // density adjoint mesh [B][nm^3]
  Vec3* g_out;         // [B * Np^3], id order
  int nm, log_nm, total;
  float scale, mass;
};

__global__ __launch_bounds__(TB) void adjoint_positions_kernel(AdjPosArgs a) {
  const int j = xcd_block(blockIdx.x, gridDim.x) * TB + threadIdx.x;
  if (j >= a.total) return;
  const uint32_t key = a.keys[j];
  const Vec3 fr = a.frac[j];
  const int nm = a.nm, lg = a.log_nm;
  const uint32_t item = key >> (3 * lg);
  const uint32_t i0[3] = {(key >> (2 * lg)) & (uint32_t)(nm - 1), (key >> lg) & (uint32_t)(nm - 1),
                          key & (uint32_t)(nm - 1)};
  const uint32_t i1[3] = {(i0[0] + 1) & (uint32_t)(nm - 1), (i0[1] + 1) & (uint32_t)(nm - 1),
                          (i0[2] + 1) & (uint32_t)(nm - 1)};
  const float f[3] = {fr.x, fr.y, fr.z};
  const size_t cells = (size_t)1 << (3 * lg);
  float fb[3] = {0.f, 0.f, 0.f};
  if (a.fbar) {
    const Vec3 v = a.fbar[j];
    fb[0] = v.x;
    fb[1] = v.y;
    fb[2] = v.z;
  }
  const Vec3* F = a.F ? a.F + (size_t)item * cells : nullptr;
  const float* D = a.dbar + (size_t)item * cells;
  const float s = a.scale;
  float gx = 0.f, gy = 0.f, gz = 0.f;
#pragma unroll
  for (int o = 0; o < 8; ++o) {
    const int ox = o >> 2, oy = (o >> 1) & 1, oz = o & 1;
    const float wx = ox ? f[0] : 1.f - f[0];
    const float wy = oy ? f[1] : 1.f - f[1];
    const float wz = oz ? f[2] : 1.f - f[2];
    const float dx = ox ? s : -s, dy = oy ? s : -s, dz = oz ? s : -s;
    const uint32_t ci = ((ox ? i1[0] : i0[0]) * (uint32_t)nm + (oy ? i1[1] : i0[1])) * (uint32_t)nm +
                        (oz ? i1[2] : i0[2]);
    float v = a.mass * D[ci];
    if (F) {
      const Vec3 fv = F[ci];
      v += fb[0] * fv.x + fb[1] * fv.y + fb[2] * fv.z;
    }
    gx += dx * wy * wz * v;
    gy += wx * dy * wz * v;
    gz += wx * wy * dz * v;
  }
  a.g_out[a.ids[j]] = Vec3{gx, gy, gz};
}

struct AdjArgs {
  float* xbar;          // in: xbar_{i+1}; out: xbar_i
  float* pbar;          // in: pbar_{i+1/2}; out: pbar_{i-1/2}
  const Vec3* gpos;   // position gradient of the step (id order)
  int log_np3, total;
  float kick, drift;
  int final_mode;       // 1: xbar = gpos, pbar = 0
  Vec3* vnext;        // nullable: kick' * (pbar_new + drift' * xbar_new) for the next
  float kick_next, drift_next;  // reverse step (its adjoint paint values)
  const uint32_t* vperm;  // nullable: sorted position of each particle in the next reverse
                          // step's sort (vnext is then written in that sort order)
};

// Step adjoint (reverse of kick then drift), with the position gradient g from above:
//   pbar' = pbar + drift * xbar;  xbar' = xbar + g
__global__ __launch_bounds__(TB) void adjoint_update_kernel(AdjArgs a) {
  const int g = xcd_block(blockIdx.x, gridDim.x) * TB + threadIdx.x;
  if (g >= a.total) return;
  const size_t np3 = (size_t)1 << a.log_np3;
  const int item = g >> a.log_np3;
  const size_t id = g & (np3 - 1);
  const size_t pi = (size_t)item * 3 * np3 + id;
  float pb[3] = {0.f, 0.f, 0.f}, xb[3] = {0.f, 0.f, 0.f};
  if (!a.final_mode) {
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      xb[q] = a.xbar[pi + q * np3];
      pb[q] = a.pbar[pi + q * np3] + a.drift * xb[q];
    }
  }
  const Vec3 gp = a.gpos[g];
  const float xn[3] = {xb[0] + gp.x, xb[1] + gp.y, xb[2] + gp.z};
  a.xbar[pi] = xn[0];
  a.xbar[pi + np3] = xn[1];
  a.xbar[pi + 2 * np3] = xn[2];
  a.pbar[pi] = pb[0];
  a.pbar[pi + np3] = pb[1];
  a.pbar[pi + 2 * np3] = pb[2];
  if (a.vnext)
    a.vnext[a.vperm ? a.vperm[g] : (uint32_t)g] =
        Vec3{a.kick_next * (pb[0] + a.drift_next * xn[0]),
             a.kick_next * (pb[1] + a.drift_next * xn[1]),
             a.kick_next * (pb[2] + a.drift_next * xn[2])};
}

// Lagrangian start: x0 = wrap(q + D0 Psi + c2x Psi2), p0 = Gp0 Psi + c2p Psi2 (Psi2 only at
// second order); q = idx * (box/np) + box / (2 nm).
__global__ __launch_bounds__(TB) void za_init_kernel(const float* __restrict__ psi,
                                                     const float* __restrict__ psi2, int np,
                                                     int log_np3, int total, double box,
                                                     double half_cell, double D0, float Gp0,
                                                     double c2x, float c2p,
                                                     double* __restrict__ x, float* __restrict__ p,
                                                     uint32_t* __restrict__ keys,
                                                     Vec3* __restrict__ frac, int key_nm,
                                                     double key_scale) {
  const int g = blockIdx.x * TB + threadIdx.x;
  if (g >= total) return;
  const size_t np3 = (size_t)1 << log_np3;
  const int item = g >> log_np3;
  const size_t id = g & (np3 - 1);
  const size_t pi = (size_t)item * 3 * np3 + id;
  const int idx[3] = {(int)(id / ((size_t)np * np)), (int)((id / np) % np), (int)(id % np)};
  const double dq = box / (double)np;
  double xn[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const float ps = psi[pi + q * np3];
    const float ps2 = psi2 ? psi2[pi + q * np3] : 0.f;
    const double q0 = (double)idx[q] * dq + half_cell;
    xn[q] = wrap_box(q0 + D0 * (double)ps + c2x * (double)ps2, box);
    x[pi + q * np3] = xn[q];
    p[pi + q * np3] = Gp0 * ps + c2p * ps2;
  }
  Vec3 f;
  keys[g] = key_frac(xn, key_scale, key_nm, item, &f);
  frac[g] = f;
}

}  // namespace

// ================================================================ host launchers
size_t sort_scratch_bytes(int n, int key_bits) {
  const int passes = (key_bits + 8) / 9;
  const int D = (key_bits + passes - 1) / passes;
  const size_t nb = (size_t)((n + SORT_TILE - 1) / SORT_TILE);
  const size_t hist = nb << D;
  // keys/ids ping-pong buffers (2 x n), histogram, offsets, digit totals
  return (2 * (size_t)n + 2 * hist + ((size_t)1 << D) + 64) * sizeof(uint32_t);
}

template <int D>
static void sort_pass(const uint32_t* kin, const uint32_t* iin, uint32_t* kout, uint32_t* iout,
                      int n, int shift, uint32_t* hist, uint32_t* offs, uint32_t* dtot,
                      const Vec3* pin, Vec3* pout, uint32_t* inv, hipStream_t s,
                      const ScatterProbe* probe) {
  const int nb = (n + SORT_TILE - 1) / SORT_TILE;
  radix_hist_kernel<D><<<nb, TB, 0, s>>>(kin, n, shift, hist);
  digit_scan_kernel<<<1 << D, TB, 0, s>>>(hist, nb, offs, dtot);
  if (probe) {
    // keys (and ids, unless the identity) in, keys and ids out, the payload gathered and
    // written, the inverse permutation written
    const double per = (iin ? 16.0 : 12.0) + (pout ? 24.0 : 0.0) + (inv ? 4.0 : 0.0);
    probe->before(probe->arg, per * n);
  }
  radix_scatter_kernel<D><<<nb, SORT_TB, 0, s>>>(kin, iin, n, shift, offs, dtot, kout, iout, pin,
                                                  pout, inv);
  if (probe) probe->after(probe->arg);
}

// Sorts keys (in place semantics: keys_io holds the input; on return `keys_sorted`
// and `ids_sorted` hold the (key, id) order). Payload starts as the identity.
void launch_sort(uint32_t* keys_io, int n, int key_bits, uint32_t* keys_sorted,
                 uint32_t* ids_sorted, void* scratch, const Vec3* pay_in, Vec3* pay_out,
                 hipStream_t s, uint32_t* inv, const ScatterProbe* probe) {
  const int passes = (key_bits + 8) / 9;
  const int D = (key_bits + passes - 1) / passes;
  const int nb = (n + SORT_TILE - 1) / SORT_TILE;
  const size_t hn = (size_t)nb << D;
  uint32_t* w = (uint32_t*)scratch;
  uint32_t* ka = w;
  uint32_t* ia = ka + n;
  uint32_t* hist = ia + n;
  uint32_t* offs = hist + hn;
  uint32_t* dtot = offs + hn;
  const uint32_t* kin = keys_io;
  const uint32_t* iin = nullptr;
  for (int p = 0; p < passes; ++p) {
    // last pass lands in the caller's output arrays
    const bool last = p == passes - 1;
    const bool to_a = ((passes - 1 - p) & 1) == 1;
    uint32_t* ko = last ? keys_sorted : (to_a ? ka : keys_sorted);
    uint32_t* io = last ? ids_sorted : (to_a ? ia : ids_sorted);
    const int shift = p * D;
    switch (D) {
#define CASE(DD) \
  case DD:                                                                                  \
    sort_pass<DD>(kin, iin, ko, io, n, shift, hist, offs, dtot, last ? pay_in : nullptr,      \
                  last ? pay_out : nullptr, last ? inv : nullptr, s, probe);                   \
    break;
      CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8) CASE(9)
#undef CASE
      default: break;
    }
    kin = ko;
    iin = io;
  }
}

void launch_row_start(const uint32_t* keys_sorted, int n, int log_nm, int rows,
                      uint32_t* row_start, hipStream_t s) {
  row_start_kernel<<<(n + 1 + TB - 1) / TB, TB, 0, s>>>(keys_sorted, n, log_nm, rows, row_start);
}

void launch_keys(const double* x, int log_np3, int total, double scale, int nm, uint32_t* keys,
                 Vec3* frac, hipStream_t s) {
  keys_kernel<<<(total + TB - 1) / TB, TB, 0, s>>>(x, log_np3, total, scale, nm, keys, frac);
}

// Rows per wave (see PMR_PAINT_LDS_FLOATS).
static int paint_ty(int nm, int C) {
  int ty = PMR_PAINT_LDS_FLOATS / (nm * C);
  if (ty > PMR_PAINT_TY_MAX) ty = PMR_PAINT_TY_MAX;
  if (ty > nm / 2) ty = nm / 2;  // TY + 1 distinct source rows per run
  int p = 1;
  while (p * 2 <= ty) p *= 2;
  return p;
}

template <int C, int TY>
static void paint_launch(const PaintArgs& a, int batch, hipStream_t s) {
  const int waves = batch * a.nm * (a.nm / TY);
  const size_t lds = (size_t)(TB / 64) * TY * C * a.nm * sizeof(float);
  paint_kernel<C, TY><<<waves / (TB / 64), TB, lds, s>>>(a);
}

template <int C>
static void paint_dispatch(const PaintArgs& a, int batch, hipStream_t s) {
  switch (paint_ty(a.nm, C)) {
    case 1: paint_launch<C, 1>(a, batch, s); break;
    case 2: paint_launch<C, 2>(a, batch, s); break;
    case 4: paint_launch<C, 4>(a, batch, s); break;
    case 8: paint_launch<C, 8>(a, batch, s); break;
    default: paint_launch<C, 16>(a, batch, s); break;
  }
}

void launch_stream_frac(const uint32_t* ids, const double* x, int total, int log_np3, int nm,
                        double box, Vec3* frac, hipStream_t s) {
  stream_frac_kernel<<<(total + TB - 1) / TB, TB, 0, s>>>(ids, x, total, log_np3,
                                                          (double)nm / box, nm, frac);
}

void launch_stream_gather(const uint32_t* ids, const Vec3* src, int total, Vec3* dst,
                          hipStream_t s) {
  stream_gather_kernel<<<(total + TB - 1) / TB, TB, 0, s>>>(ids, src, total, dst);
}

void launch_paint_mass(const uint32_t* keys, const Vec3* frac, const uint32_t* row_start,
                       int batch, int nm, float mass, float bias, float* out, hipStream_t s) {
  PaintArgs a{};
  a.keys = keys;
  a.frac = frac;
  a.row_start = row_start;
  a.nm = nm;
  int l = 0;
  while ((1 << l) < nm) ++l;
  a.log_nm = l;
  a.mass = mass;
  a.bias = bias;
  a.out = out;
  paint_dispatch<1>(a, batch, s);
}

void launch_kick_drift(const double* x, double* x_next, float* p, const Vec3* F, uint32_t* keys,
                       Vec3* frac, int batch, int log_np3, int nm, double box, float kick,
                       double drift, int key_nm, hipStream_t s) {
  StepArgs a{};
  a.frac = frac;
  a.x = x;
  a.x_next = x_next;
  a.p = p;
  a.F = F;
  a.keys = keys;
  a.log_np3 = log_np3;
  a.nm = nm;
  a.total = batch << log_np3;
  a.scale = (double)nm / box;
  a.box = box;
  a.kick = kick;
  a.drift = drift;
  a.key_nm = key_nm;
  a.key_scale = (double)key_nm / box;
  kick_drift_kernel<<<(a.total + TB - 1) / TB, TB, 0, s>>>(a);
}

void launch_adjoint_positions(const uint32_t* keys, const Vec3* frac, const Vec3* fbar,
                              const uint32_t* ids, const Vec3* F, const float* dbar, int total,
                              int nm, double box, float mass, Vec3* g_out, hipStream_t s) {
  AdjPosArgs a{};
  a.keys = keys;
  a.frac = frac;
  a.fbar = fbar;
  a.ids = ids;
  a.F = F;
  a.dbar = dbar;
  a.g_out = g_out;
  a.nm = nm;
  int l = 0;
  while ((1 << l) < nm) ++l;
  a.log_nm = l;
  a.total = total;
  a.scale = (float)((double)nm / box);
  a.mass = mass;
  adjoint_positions_kernel<<<(total + TB - 1) / TB, TB, 0, s>>>(a);
}

void launch_adjoint_update(float* xbar, float* pbar, const Vec3* gpos, int batch, int log_np3,
                           float kick, float drift, int final_mode, Vec3* vnext, float kick_next,
                           float drift_next, const uint32_t* vperm, hipStream_t s) {
  AdjArgs a{};
  a.xbar = xbar;
  a.pbar = pbar;
  a.gpos = gpos;
  a.log_np3 = log_np3;
  a.total = batch << log_np3;
  a.kick = kick;
  a.drift = drift;
  a.final_mode = final_mode;
  a.vnext = vnext;
  a.kick_next = kick_next;
  a.drift_next = drift_next;
  a.vperm = vperm;
  adjoint_update_kernel<<<(a.total + TB - 1) / TB, TB, 0, s>>>(a);
}

void launch_za_init(const float* psi, const float* psi2, int batch, int np, int log_np3,
                    double box, double half_cell, double D0, float Gp0, double c2x, float c2p,
                    double* x, float* p, uint32_t* keys, Vec3* frac, int key_nm, hipStream_t s) {
  const int total = batch << log_np3;
  za_init_kernel<<<(total + TB - 1) / TB, TB, 0, s>>>(psi, psi2, np, log_np3, total, box,
                                                       half_cell, D0, Gp0, c2x, c2p, x, p, keys,
                                                       frac, key_nm, (double)key_nm / box);
}

}  // namespace pmr
