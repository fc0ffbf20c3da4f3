// The paper's two-network halo model (Sec. 2.1: model = NNp x NNm; Sec. 2.3: architecture;
// Sec. 2.2: features) and its input gradient, on the output mesh.
//
// Per voxel v with feature fields f = (delta_0, delta_R1, delta_R1 - delta_R2):
//   NNp: the 81 values of f on the 3 x 3 x 3 neighbourhood -> 50 -> 30 (ReLU) -> y,
//        pos = logistic(y, a) = 1 / (1 + exp(-a y))            (the position mask)
//   NNm: f(v) -> 20 -> 10 (ELU) -> m, linear                    (the mass)
//   mass = pos * m.
// Adjoint (weights frozen): with Mbar the mass adjoint, ybar = Mbar m a pos (1 - pos) and
// mbar = Mbar pos are pushed back through the layers; the position network's input adjoint
// u (81 per voxel) belongs to the neighbours, so it is written out and a second kernel sums,
// for each voxel, the 27 entries that point at it: fbar_c(y) = sum_o u_{c,o}(y - d_o).
//
// One thread per voxel, FP32 on the vector units. The hidden loop runs over the 50 first-
// layer neurons: each neuron's 81-term dot product is followed at once by its contribution
// to the 30 second-layer sums (and, in the adjoint, its share of the 81 input adjoints), so
// no per-neuron array is indexed at run time; the layer-1 ReLU signs are kept as a 64-bit
// mask. Weights are read at wave-uniform addresses (scalar loads).
#include "../../include/pmr.h"
#include "pmr_internal.h"

namespace pmr {
namespace {

constexpr int TB = 256;
constexpr int NP1 = 50, NP2 = 30, NF = 81, NM1 = 20, NM2 = 10;

// Prepared weight block (floats). Rows of the position network's first layer are padded
// to 84 and its second layer is stored transposed ([j][k], rows padded to 32), so that the
// hidden loop reads contiguous rows.
struct H2 {
  static constexpr int W1 = 0;                 // [50][84]
  static constexpr int B1 = W1 + NP1 * 84;     // [50] (+2)
  static constexpr int W2T = B1 + 52;          // [50][32]
  static constexpr int B2 = W2T + NP1 * 32;    // [32]
  static constexpr int W3 = B2 + 32;           // [32]
  static constexpr int B3 = W3 + 32;           // [1] (+3)
  static constexpr int M1 = B3 + 4;            // [20][4]: W1m[u][0..2], b1m[u]
  static constexpr int M2 = M1 + NM1 * 4;      // [10][20]
  static constexpr int MB2 = M2 + NM2 * NM1;   // [10] (+2)
  static constexpr int MW3 = MB2 + 12;         // [10] (+2)
  static constexpr int MB3 = MW3 + 12;         // [1] (+3)
  static constexpr int SIZE = MB3 + 4;
};
static_assert(H2::SIZE == HALO2_WEIGHT_FLOATS, "prepared weight block size");

// Packed user blocks -> prepared block (zero padding).
__global__ void halo2_prepare_kernel(const float* __restrict__ nnp, const float* __restrict__ nnm,
                                     float* __restrict__ w) {
  constexpr int pW1 = 0, pB1 = NP1 * NF, pW2 = pB1 + NP1, pB2 = pW2 + NP2 * NP1, pW3 = pB2 + NP2,
                pB3 = pW3 + NP2;
  constexpr int mW1 = 0, mB1 = NM1 * 3, mW2 = mB1 + NM1, mB2 = mW2 + NM2 * NM1, mW3 = mB2 + NM2,
                mB3 = mW3 + NM2;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < H2::SIZE; i += gridDim.x * blockDim.x) {
    float v = 0.f;
    if (i < H2::B1) {
      const int j = i / 84, f = i % 84;
      if (f < NF) v = nnp[pW1 + j * NF + f];
    } else if (i < H2::W2T) {
      const int j = i - H2::B1;
      if (j < NP1) v = nnp[pB1 + j];
    } else if (i < H2::B2) {
      const int j = (i - H2::W2T) / 32, k = (i - H2::W2T) % 32;
      if (k < NP2) v = nnp[pW2 + k * NP1 + j];
    } else if (i < H2::W3) {
      const int k = i - H2::B2;
      if (k < NP2) v = nnp[pB2 + k];
    } else if (i < H2::B3) {
      const int k = i - H2::W3;
      if (k < NP2) v = nnp[pW3 + k];
    } else if (i < H2::M1) {
      if (i == H2::B3) v = nnp[pB3];
    } else if (i < H2::M2) {
      const int u = (i - H2::M1) / 4, e = (i - H2::M1) % 4;
      v = e < 3 ? nnm[mW1 + u * 3 + e] : nnm[mB1 + u];
    } else if (i < H2::MB2) {
      v = nnm[mW2 + (i - H2::M2)];
    } else if (i < H2::MW3) {
      const int q = i - H2::MB2;
      if (q < NM2) v = nnm[mB2 + q];
    } else if (i < H2::MB3) {
      const int q = i - H2::MW3;
      if (q < NM2) v = nnm[mW3 + q];
    } else if (i == H2::MB3) {
      v = nnm[mB3];
    }
    w[i] = v;
  }
}

__device__ __forceinline__ float elu_f(float z) { return z > 0.f ? z : expm1f(z); }

struct Vox {
  size_t base;  // first voxel of the item
  int ix, iy, iz;
};

__device__ __forceinline__ Vox vox(size_t v, int log_n) {
  const size_t n3 = (size_t)1 << (3 * log_n);
  Vox r;
  r.base = v & ~(n3 - 1);
  const size_t l = v & (n3 - 1);
  const int m = (1 << log_n) - 1;
  r.ix = (int)(l >> (2 * log_n));
  r.iy = (int)(l >> log_n) & m;
  r.iz = (int)l & m;
  return r;
}

__device__ __forceinline__ size_t nbr(const Vox& p, int log_n, int dx, int dy, int dz) {
  const int m = (1 << log_n) - 1;
  return p.base + ((size_t)((p.ix + dx) & m) << (2 * log_n)) + ((size_t)((p.iy + dy) & m) << log_n) +
         (size_t)((p.iz + dz) & m);
}

// BWD = false: mass = pos * m. BWD = true: with mbar given, writes the position network's
// input adjoint u [B][81][n^3] and the mass network's input adjoint as (g0, g12, g2) =
// (fbar_0, fbar_1 + fbar_2, fbar_2).
template <bool BWD>
__global__ __launch_bounds__(TB) void halo2_kernel(const float* __restrict__ d0,
                                                   const float* __restrict__ d1,
                                                   const float* __restrict__ d2, int log_n,
                                                   size_t total, const float* __restrict__ w,
                                                   const double* __restrict__ prm,
                                                   const float* __restrict__ mbar,
                                                   float* __restrict__ mass,
                                                   float* __restrict__ U, float* __restrict__ g0,
                                                   float* __restrict__ g12,
                                                   float* __restrict__ g2) {
  const size_t v = (size_t)blockIdx.x * TB + threadIdx.x;
  if (v >= total) return;
  const Vox p = vox(v, log_n);
  const size_t n3 = (size_t)1 << (3 * log_n);
  const size_t item = v >> (3 * log_n);
  float x[NF];
#pragma unroll
  for (int o = 0; o < 27; ++o) {
    const size_t q = nbr(p, log_n, o / 9 - 1, (o / 3) % 3 - 1, o % 3 - 1);
    const float r1 = d1[q];
    x[o] = d0[q];
    x[27 + o] = r1;
    x[54 + o] = r1 - d2[q];
  }
  // position network, forward
  float a2[NP2];
#pragma unroll
  for (int k = 0; k < NP2; ++k) a2[k] = w[H2::B2 + k];
  uint64_t mask = 0;
#pragma unroll 1
  for (int j = 0; j < NP1; ++j) {
    const float* r = w + H2::W1 + j * 84;
    float t = w[H2::B1 + j];
#pragma unroll
    for (int f = 0; f < NF; ++f) t = fmaf(r[f], x[f], t);
    if (t > 0.f) {
      mask |= (uint64_t)1 << j;
    } else {
      t = 0.f;
    }
    const float* c = w + H2::W2T + j * 32;
#pragma unroll
    for (int k = 0; k < NP2; ++k) a2[k] = fmaf(c[k], t, a2[k]);
  }
  float y = w[H2::B3];
#pragma unroll
  for (int k = 0; k < NP2; ++k) y = fmaf(w[H2::W3 + k], fmaxf(a2[k], 0.f), y);
  const float a = (float)prm[item * NPRM + 6];
  const float pos = 1.f / (1.f + expf(-a * y));
  // mass network, forward
  const float x3[3] = {x[13], x[40], x[67]};
  float e1[NM1];
#pragma unroll
  for (int u = 0; u < NM1; ++u) {
    const float* r = w + H2::M1 + 4 * u;
    e1[u] = elu_f(fmaf(r[0], x3[0], fmaf(r[1], x3[1], fmaf(r[2], x3[2], r[3]))));
  }
  float e2[NM2];
  float mm = w[H2::MB3];
#pragma unroll
  for (int q = 0; q < NM2; ++q) {
    float z = w[H2::MB2 + q];
#pragma unroll
    for (int u = 0; u < NM1; ++u) z = fmaf(w[H2::M2 + q * NM1 + u], e1[u], z);
    e2[q] = elu_f(z);
    mm = fmaf(w[H2::MW3 + q], e2[q], mm);
  }
  if constexpr (!BWD) {
    mass[v] = pos * mm;
    return;
  } else {
    const float mb = mbar[v];
    // position network, adjoint
    const float yb = mb * mm * a * pos * (1.f - pos);
    float a2b[NP2];
#pragma unroll
    for (int k = 0; k < NP2; ++k) a2b[k] = a2[k] > 0.f ? w[H2::W3 + k] * yb : 0.f;
    float u[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) u[f] = 0.f;
#pragma unroll 1
    for (int j = 0; j < NP1; ++j) {
      const float* c = w + H2::W2T + j * 32;
      float g = 0.f;
#pragma unroll
      for (int k = 0; k < NP2; ++k) g = fmaf(c[k], a2b[k], g);
      g = ((mask >> j) & 1) ? g : 0.f;
      const float* r = w + H2::W1 + j * 84;
#pragma unroll
      for (int f = 0; f < NF; ++f) u[f] = fmaf(r[f], g, u[f]);
    }
    float* uo = U + item * NF * n3 + (v & (n3 - 1));
#pragma unroll
    for (int f = 0; f < NF; ++f) uo[(size_t)f * n3] = u[f];
    // mass network, adjoint (ELU'(z) = 1 for z > 0, else exp(z) = ELU(z) + 1)
    const float mbm = mb * pos;
    float e1b[NM1];
#pragma unroll
    for (int s = 0; s < NM1; ++s) e1b[s] = 0.f;
#pragma unroll
    for (int q = 0; q < NM2; ++q) {
      const float d = e2[q] > 0.f ? 1.f : e2[q] + 1.f;
      const float zb = w[H2::MW3 + q] * mbm * d;
#pragma unroll
      for (int s = 0; s < NM1; ++s) e1b[s] = fmaf(w[H2::M2 + q * NM1 + s], zb, e1b[s]);
    }
    float fb0 = 0.f, fb1 = 0.f, fb2 = 0.f;
#pragma unroll
    for (int s = 0; s < NM1; ++s) {
      const float d = e1[s] > 0.f ? 1.f : e1[s] + 1.f;
      const float zb = e1b[s] * d;
      const float* r = w + H2::M1 + 4 * s;
      fb0 = fmaf(r[0], zb, fb0);
      fb1 = fmaf(r[1], zb, fb1);
      fb2 = fmaf(r[2], zb, fb2);
    }
    g0[v] = fb0;
    g12[v] = fb1 + fb2;
    g2[v] = fb2;
  }
}

// fbar_c(y) = sum_o u_{c,o}(y - d_o), added to (g0, g12, g2).
__global__ __launch_bounds__(TB) void halo2_stencil_adj_kernel(const float* __restrict__ U,
                                                               int log_n, size_t total,
                                                               float* __restrict__ g0,
                                                               float* __restrict__ g12,
                                                               float* __restrict__ g2) {
  const size_t v = (size_t)blockIdx.x * TB + threadIdx.x;
  if (v >= total) return;
  const Vox p = vox(v, log_n);
  const size_t n3 = (size_t)1 << (3 * log_n);
  const float* ub = U + (v >> (3 * log_n)) * NF * n3;
  float s[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int o = 0; o < 27; ++o) {
    const size_t q = nbr(p, log_n, 1 - o / 9, 1 - (o / 3) % 3, 1 - o % 3) - p.base;
#pragma unroll
    for (int c = 0; c < 3; ++c) s[c] += ub[(size_t)(c * 27 + o) * n3 + q];
  }
  g0[v] += s[0];
  g12[v] += s[1] + s[2];
  g2[v] += s[2];
}

}  // namespace

void launch_halo2_prepare(const float* nnp, const float* nnm, float* w, hipStream_t s) {
  halo2_prepare_kernel<<<(H2::SIZE + TB - 1) / TB, TB, 0, s>>>(nnp, nnm, w);
}

void launch_halo2_fwd(const float* d0, const float* d1, const float* d2, int log_n, size_t total,
                      const float* w, const double* prm, float* mass, hipStream_t s) {
  halo2_kernel<false><<<(unsigned)((total + TB - 1) / TB), TB, 0, s>>>(
      d0, d1, d2, log_n, total, w, prm, nullptr, mass, nullptr, nullptr, nullptr, nullptr);
}

void launch_halo2_bwd(const float* d0, const float* d1, const float* d2, int log_n, size_t total,
                      const float* w, const double* prm, const float* mbar, float* U, float* g0,
                      float* g12, float* g2, hipStream_t s) {
  halo2_kernel<true><<<(unsigned)((total + TB - 1) / TB), TB, 0, s>>>(
      d0, d1, d2, log_n, total, w, prm, mbar, nullptr, U, g0, g12, g2);
}

void launch_halo2_stencil_adj(const float* U, int log_n, size_t total, float* g0, float* g12,
                              float* g2, hipStream_t s) {
  halo2_stencil_adj_kernel<<<(unsigned)((total + TB - 1) / TB), TB, 0, s>>>(U, log_n, total, g0,
                                                                            g12, g2);
}

}  // namespace pmr
