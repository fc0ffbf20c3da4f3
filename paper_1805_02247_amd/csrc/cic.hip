// Particles: cell keys, the stable (cell, id) sort, cloud-in-cell paint and readout,
// kick/drift and their adjoints.
//
// Particle state is kept in Lagrangian (id) order: id = (i*Np + j)*Np + k for the lattice
// site (i, j, k), which keeps neighbouring ids close in space through the evolution, so
// the per-particle gathers below stay cache friendly without moving the state.
// Positions are FP64 [B][3][Np^3]; momenta and adjoints FP32 [B][3][Np^3].
//
// Keys carry the batch item: key = item*Nm^3 + (ix*Nm + iy)*Nm + iz, with (ix, iy, iz)
// the lower CIC corner computed in FP64. The cell sort (sort.hip) gives the unique
// (key, id) order; rows (item, ix, iy) are then contiguous and `row_start` indexes them.
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
  const Vec3 v = src[ids[j]];
  // non-temporal: the stream is read once, by the paint that follows the whole pass
  __builtin_nontemporal_store(v.x, &dst[j].x);
  __builtin_nontemporal_store(v.y, &dst[j].y);
  __builtin_nontemporal_store(v.z, &dst[j].z);
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
  const float* p_in;  // momenta before the kick (usually p_out: updated in place)
  float* p_out;       // momenta after the kick
  float* p_ck;        // nullable: a second copy of p_out (the checkpoint of the next step)
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

// First particle of block L when the lattice rows (item, i, j, :) are visited in patches of
// 2^logP x 2^logP rows (j fastest within a patch, then i, then the patch): a lattice row
// holds np / TB whole blocks, and the force-mesh rows a patch reads overlap those of its
// neighbours in both i and j, so one XCD's blocks in flight share more of their corner
// rows in L2 than with the plain row order. A bijection of the block indices, so the
// result does not depend on it.
__device__ __forceinline__ int patch_block_start(int L, int log_np, int logP) {
  const int np = 1 << log_np;
  const int bpr = np / TB;
  const int kb = L % bpr;
  int r = L / bpr;
  const int item = r >> (2 * log_np);
  r &= (1 << (2 * log_np)) - 1;
  const int P = 1 << logP, tiles = np >> logP;
  const int jj = r & (P - 1);
  r >>= logP;
  const int ii = r & (P - 1);
  r >>= logP;
  const int pj = r % tiles, pi = r / tiles;
  const int i = pi * P + ii, j = pj * P + jj;
  return (item << (3 * log_np)) + ((i * np + j) << log_np) + kb * TB;
}
constexpr int KD_PATCH_LOG = 5;  // 32 x 32 lattice rows per patch

// p += kick * F(x_i);  x_{i+1} = wrap(x_i + drift * p);  key(x_{i+1})
__global__ __launch_bounds__(TB) void kick_drift_kernel(StepArgs a) {
  const int L = xcd_block(blockIdx.x, gridDim.x);
  const int log_np = a.log_np3 / 3;
  const int g = ((1 << log_np) >= TB && log_np >= KD_PATCH_LOG)
                    ? patch_block_start(L, log_np, KD_PATCH_LOG) + threadIdx.x
                    : L * TB + threadIdx.x;
  if (g >= a.total) return;
  const size_t np3 = (size_t)1 << a.log_np3;
  const int item = g >> a.log_np3;
  const size_t id = g & (np3 - 1);
  const size_t pi = (size_t)item * 3 * np3 + id;
  // the particle's own streams are read once: non-temporal loads, so that the force-mesh
  // corners stay in the caches (likewise the sorted streams of the adjoint gather)
  double xyz[3] = {__builtin_nontemporal_load(a.x + pi),
                   __builtin_nontemporal_load(a.x + pi + np3),
                   __builtin_nontemporal_load(a.x + pi + 2 * np3)};
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
  // The outputs go out with non-temporal stores, so that they do not displace the force
  // mesh the corner gathers read from the caches: x and p are read again only a step later,
  // the keys and fractions by the sort in another order (measured 2-5% faster per launch at
  // 256^3/512^3 with the force mesh written the same way; bit for bit the same results).
  double xn[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const float pq = __builtin_nontemporal_load(a.p_in + pi + q * np3) + a.kick * fa[q];
    __builtin_nontemporal_store(pq, a.p_out + pi + q * np3);
    if (a.p_ck) __builtin_nontemporal_store(pq, a.p_ck + pi + q * np3);
    xn[q] = wrap_box(xyz[q] + a.drift * (double)pq, a.box);
    __builtin_nontemporal_store(xn[q], a.x_next + pi + q * np3);
  }
  if (a.keys) {
    Vec3 f;
    __builtin_nontemporal_store(key_frac(xn, a.key_scale, a.key_nm, item, &f), a.keys + g);
    __builtin_nontemporal_store(f.x, &a.frac[g].x);
    __builtin_nontemporal_store(f.y, &a.frac[g].y);
    __builtin_nontemporal_store(f.z, &a.frac[g].z);
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

// WF: the force term is present (F and fbar set). A compile-time switch rather than a
// per-corner test of F, so that the 16 corner loads are issued together instead of each
// waiting behind a branch.
template <bool WF>
__global__ __launch_bounds__(TB) void adjoint_positions_kernel(AdjPosArgs a) {
  const int j = xcd_block(blockIdx.x, gridDim.x) * TB + threadIdx.x;
  if (j >= a.total) return;
  const uint32_t key = __builtin_nontemporal_load(a.keys + j);
  const Vec3 fr = Vec3{__builtin_nontemporal_load(&a.frac[j].x),
                       __builtin_nontemporal_load(&a.frac[j].y),
                       __builtin_nontemporal_load(&a.frac[j].z)};
  const int nm = a.nm, lg = a.log_nm;
  const uint32_t item = key >> (3 * lg);
  const uint32_t i0[3] = {(key >> (2 * lg)) & (uint32_t)(nm - 1), (key >> lg) & (uint32_t)(nm - 1),
                          key & (uint32_t)(nm - 1)};
  const uint32_t i1[3] = {(i0[0] + 1) & (uint32_t)(nm - 1), (i0[1] + 1) & (uint32_t)(nm - 1),
                          (i0[2] + 1) & (uint32_t)(nm - 1)};
  const float f[3] = {fr.x, fr.y, fr.z};
  const size_t cells = (size_t)1 << (3 * lg);
  float fb[3] = {0.f, 0.f, 0.f};
  if (WF) {
    const Vec3 v = a.fbar[j];
    fb[0] = v.x;
    fb[1] = v.y;
    fb[2] = v.z;
  }
  const Vec3* F = WF ? a.F + (size_t)item * cells : nullptr;
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
    if (WF) {
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
                                                     float* __restrict__ p_ck,
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
    if (p_ck) p_ck[pi + q * np3] = Gp0 * ps + c2p * ps2;
  }
  Vec3 f;
  keys[g] = key_frac(xn, key_scale, key_nm, item, &f);
  frac[g] = f;
}

}  // namespace

// ================================================================ host launchers
void launch_keys(const double* x, int log_np3, int total, double scale, int nm, uint32_t* keys,
                 Vec3* frac, hipStream_t s) {
  keys_kernel<<<(total + TB - 1) / TB, TB, 0, s>>>(x, log_np3, total, scale, nm, keys, frac);
}

// Rows per wave: the tuned value when set and valid, else the default rule (see
// PMR_PAINT_LDS_FLOATS).
static int paint_ty(int nm, int C) {
  const int want = get_paint_rows(nm, C);
  if (want > 0 && want <= nm / 2 && (size_t)(TB / 64) * want * C * nm * 4 <= 64 * 1024)
    return want;
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

void launch_kick_drift(const double* x, double* x_next, const float* p_in, float* p,
                       float* p_ck, const Vec3* F, uint32_t* keys, Vec3* frac, int batch,
                       int log_np3, int nm, double box, float kick, double drift, int key_nm,
                       hipStream_t s) {
  StepArgs a{};
  a.frac = frac;
  a.x = x;
  a.x_next = x_next;
  a.p_in = p_in ? p_in : p;
  a.p_out = p;
  a.p_ck = p_ck;
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
  if (a.F && a.fbar)
    adjoint_positions_kernel<true><<<(total + TB - 1) / TB, TB, 0, s>>>(a);
  else
    adjoint_positions_kernel<false><<<(total + TB - 1) / TB, TB, 0, s>>>(a);
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
                    double* x, float* p, float* p_ck, uint32_t* keys, Vec3* frac, int key_nm,
                    hipStream_t s) {
  const int total = batch << log_np3;
  za_init_kernel<<<(total + TB - 1) / TB, TB, 0, s>>>(psi, psi2, np, log_np3, total, box,
                                                       half_cell, D0, Gp0, c2x, c2p, x, p, p_ck,
                                                       keys, frac, key_nm, (double)key_nm / box);
}

}  // namespace pmr
