// The paper's two-network halo model (Sec. 2: model = NNp x NNm; Sec. 2.1: architecture;
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
// The position network's four products (forward 81 -> 50 -> 30, adjoint 30 -> 50 -> 81) run
// on the matrix cores in FP32; the forward keeps pos and the ReLU signs for the adjoint, so
// the adjoint runs only the two transposed products. The small mass network runs one thread
// per voxel on the vector units, in its own kernel, with pos and m passed through a
// [2][B][n^3] buffer.
#include "../../include/pmr.h"
#include "pmr_internal.h"

namespace pmr {
namespace {

constexpr int TB = 256;
constexpr int NP1 = 50, NP2 = 30, NF = 81, NM1 = 20, NM2 = 10;

// Prepared weight block (floats): the position network's biases and output row, the mass
// network, then the matrix-core operand fragments of the position network's four products
// (described below), each [tile][k step][64 lanes].
struct H2 {
  static constexpr int B1 = 0;                 // [50] (+14)
  static constexpr int B2 = B1 + 64;           // [30] (+2)
  static constexpr int W3 = B2 + 32;           // [30] (+2)
  static constexpr int B3 = W3 + 32;           // [1] (+3)
  static constexpr int M1 = B3 + 4;            // [20][4]: W1m[u][0..2], b1m[u]
  static constexpr int M2 = M1 + NM1 * 4;      // [10][20]
  static constexpr int MB2 = M2 + NM2 * NM1;   // [10] (+2)
  static constexpr int MW3 = MB2 + 12;         // [10] (+2)
  static constexpr int MB3 = MW3 + 12;         // [1] (+3)
  static constexpr int F1 = 448;               // W1:   4 x 21
  static constexpr int F2 = F1 + 4 * 21 * 64;  // W2:   2 x 16
  static constexpr int F3 = F2 + 2 * 16 * 64;  // W2^T: 4 x 8
  static constexpr int F4 = F3 + 4 * 8 * 64;   // W1^T: 6 x 16
  static constexpr int SIZE = F4 + 6 * 16 * 64;
};
static_assert(H2::MB3 + 4 <= H2::F1 && H2::F1 % 64 == 0, "fragment regions follow the plain block");
static_assert(H2::SIZE == HALO2_WEIGHT_FLOATS, "prepared weight block size");

// Matrix-core form (v_mfma_f32_16x16x4f32, FP32 in and out). Voxels are the column (N)
// dimension of every product, 16 per wavefront step; lane l holds column n = l % 16 and
// lane group g = l / 16. Operands (one float per lane per instruction):
//   A[m][k]: m = l % 16, k = l / 16;   B[k][n]: k = l / 16;   C[m][n]: m = 4 g + i (i < 4).
// Layer 1 takes, at k step kb, feature field kb / 7 at neighbourhood offset
// o = 4 (kb % 7) + g (o < 27; 81 features in 21 steps), so a lane computes 7 neighbour
// addresses and reads all three fields at each. The K slots
// of the later products are mapped onto the C layout of the product before:
//   slot(kb, g) = 16 (kb / 4) + 4 g + kb % 4,
// so one product's accumulators (tile kb / 4, element kb % 4) are the next product's B
// operand with no data movement, and the layer-1 ReLU signs sit in the lanes of the layer-1
// adjoint. Products: (1) a1 = W1 x (50 -> 4 tiles of 16, K 84); (2) a2 = W2 h1 (30 -> 2
// tiles, K 64); adjoint (3) a1bar = W2^T a2bar (4 tiles, K 32); (4) u = W1^T a1bar (81 -> 6
// tiles, K 64). Padding rows and columns are zero in the fragments.
__host__ __device__ constexpr int mx_slot(int kb, int g) { return 16 * (kb >> 2) + 4 * g + (kb & 3); }

// Packed user blocks -> prepared block (zero padding).
__global__ void halo2_prepare_kernel(const float* __restrict__ nnp, const float* __restrict__ nnm,
                                     float* __restrict__ w) {
  constexpr int pW1 = 0, pB1 = NP1 * NF, pW2 = pB1 + NP1, pB2 = pW2 + NP2 * NP1, pW3 = pB2 + NP2,
                pB3 = pW3 + NP2;
  constexpr int mW1 = 0, mB1 = NM1 * 3, mW2 = mB1 + NM1, mB2 = mW2 + NM2 * NM1, mW3 = mB2 + NM2,
                mB3 = mW3 + NM2;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < H2::SIZE; i += gridDim.x * blockDim.x) {
    float v = 0.f;
    if (i < H2::B2) {
      const int j = i - H2::B1;
      if (j < NP1) v = nnp[pB1 + j];
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
    } else if (i >= H2::F1 && i < H2::F2) {
      const int e = i - H2::F1, l = e & 63, kb = (e >> 6) % 21, mt = (e >> 6) / 21;
      const int m = 16 * mt + (l & 15), c = kb / 7, o = 4 * (kb % 7) + (l >> 4);
      if (m < NP1 && o < 27) v = nnp[pW1 + m * NF + c * 27 + o];
    } else if (i >= H2::F2 && i < H2::F3) {
      const int e = i - H2::F2, l = e & 63, kb = (e >> 6) % 16, mt = (e >> 6) / 16;
      const int m = 16 * mt + (l & 15), k = mx_slot(kb, l >> 4);
      if (m < NP2 && k < NP1) v = nnp[pW2 + m * NP1 + k];
    } else if (i >= H2::F3 && i < H2::F4) {
      const int e = i - H2::F3, l = e & 63, kb = (e >> 6) % 8, mt = (e >> 6) / 8;
      const int m = 16 * mt + (l & 15), k = mx_slot(kb, l >> 4);  // m: layer-1, k: layer-2
      if (m < NP1 && k < NP2) v = nnp[pW2 + k * NP1 + m];
    } else if (i >= H2::F4) {
      const int e = i - H2::F4, l = e & 63, kb = (e >> 6) % 16, mt = (e >> 6) / 16;
      const int m = 16 * mt + (l & 15), k = mx_slot(kb, l >> 4);  // m: feature, k: layer-1
      if (m < NF && k < NP1) v = nnp[pW1 + k * NF + m];
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

// Mass network, one thread per voxel. BWD = false: m = NNm(f) to mout, mass = pos * m.
// BWD = true: (g0, g12, g2) = the network's input adjoint for mbar * pos, as
// (fbar_0, fbar_1 + fbar_2, fbar_2) (the features' adjoint needs G_R1 (fbar_1 + fbar_2) -
// G_R2 fbar_2); ELU'(z) = 1 for z > 0, else exp(z) = ELU(z) + 1.
template <bool BWD>
__global__ __launch_bounds__(TB) void halo2_nnm_kernel(const float* __restrict__ d0,
                                                       const float* __restrict__ d1,
                                                       const float* __restrict__ d2, size_t total,
                                                       const float* __restrict__ w,
                                                       const float* __restrict__ pos,
                                                       const float* __restrict__ mbar,
                                                       float* __restrict__ mout,
                                                       float* __restrict__ mass,
                                                       float* __restrict__ g0,
                                                       float* __restrict__ g12,
                                                       float* __restrict__ g2) {
  const size_t v = (size_t)blockIdx.x * TB + threadIdx.x;
  if (v >= total) return;
  const float r1 = d1[v];
  const float x3[3] = {d0[v], r1, r1 - d2[v]};
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
    mout[v] = mm;
    mass[v] = pos[v] * mm;
  } else {
    const float mbm = mbar[v] * pos[v];
    float e1b[NM1];
#pragma unroll
    for (int u = 0; u < NM1; ++u) e1b[u] = 0.f;
#pragma unroll
    for (int q = 0; q < NM2; ++q) {
      const float d = e2[q] > 0.f ? 1.f : e2[q] + 1.f;
      const float zb = w[H2::MW3 + q] * mbm * d;
#pragma unroll
      for (int u = 0; u < NM1; ++u) e1b[u] = fmaf(w[H2::M2 + q * NM1 + u], zb, e1b[u]);
    }
    float fb0 = 0.f, fb1 = 0.f, fb2 = 0.f;
#pragma unroll
    for (int u = 0; u < NM1; ++u) {
      const float d = e1[u] > 0.f ? 1.f : e1[u] + 1.f;
      const float zb = e1b[u] * d;
      const float* r = w + H2::M1 + 4 * u;
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
  float s[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int o = 0; o < 27; ++o) {
    const size_t q = nbr(p, log_n, 1 - o / 9, 1 - (o / 3) % 3, 1 - o % 3);
    const float* uq = U + (q >> 4) * NF * 16 + (q & 15);
#pragma unroll
    for (int c = 0; c < 3; ++c) s[c] += uq[(c * 27 + o) * 16];
  }
  g0[v] += s[0];
  g12[v] += s[1] + s[2];
  g2[v] += s[2];
}

typedef float floatx4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ floatx4_t mx(float a, float b, floatx4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

constexpr int MX_WAVES = 8;  // wavefronts per workgroup

// LDS base address made to depend on `after`, so that the compiler cannot hoist a later
// product's operand reads above the product that produces `after` (they would all be live
// at once and spill).
__device__ __forceinline__ const float* lds_after(const float* base, float after) {
  int z = 0;
  asm volatile("" : "+v"(z) : "v"(after));
  return base + z;
}

// Persistent: each wavefront takes 16-voxel groups in a grid-stride loop; the operand
// fragments are staged in LDS once per workgroup (29 KB forward, 32 KB adjoint).
// Position network, forward: pos = logistic(y, a) to aux[v]; the ReLU signs of the lane's
// 16 layer-1 and 8 layer-2 neurons (C layout) to bits 0..15 and 16..23 of sgn[v][g], for
// the adjoint.
__global__ __launch_bounds__(64 * MX_WAVES) void halo2_mx_fwd_kernel(
    const float* __restrict__ d0, const float* __restrict__ d1, const float* __restrict__ d2,
    int log_n, size_t groups, const float* __restrict__ w, const double* __restrict__ prm,
    float* __restrict__ aux, uint32_t* __restrict__ sgn) {
  constexpr int NFRAG = H2::F3 - H2::F1;
  __shared__ __attribute__((aligned(16))) float sf[NFRAG];
  __shared__ float sv[H2::M1];  // b1, b2, W3, b3: read per lane group, kept close
  for (int i = threadIdx.x; i < NFRAG / 4; i += 64 * MX_WAVES)
    reinterpret_cast<float4*>(sf)[i] = reinterpret_cast<const float4*>(w + H2::F1)[i];
  for (int i = threadIdx.x; i < H2::M1; i += 64 * MX_WAVES) sv[i] = w[i];
  __syncthreads();
  const float* f1 = sf;
  const float* f2 = sf + (H2::F2 - H2::F1);
  const int l = threadIdx.x & 63, g = l >> 4, n = l & 15;
  const size_t stride = (size_t)gridDim.x * MX_WAVES;
  for (size_t G = (size_t)xcd_block(blockIdx.x, gridDim.x) * MX_WAVES + (threadIdx.x >> 6);
       G < groups; G += stride) {
    const size_t v = G * 16 + n;
    const Vox p = vox(v, log_n);
    const size_t item = v >> (3 * log_n);
    // B operands of layer 1: the three fields at offsets o = 4 kk + g of this lane's voxel
    float xb[21];
#pragma unroll
    for (int kk = 0; kk < 7; ++kk) {
      const int o = 4 * kk + g;
      float x0 = 0.f, x1 = 0.f, x2 = 0.f;
      if (o < 27) {
        const size_t q = nbr(p, log_n, o / 9 - 1, (o / 3) % 3 - 1, o % 3 - 1);
        x0 = d0[q];
        x1 = d1[q];
        x2 = x1 - d2[q];
      }
      xb[kk] = x0;
      xb[7 + kk] = x1;
      xb[14 + kk] = x2;
    }
    // (1) a1 = W1 x + b1, h1 = ReLU(a1)
    floatx4_t h1[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) h1[mt] = floatx4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < 21; ++kb)
#pragma unroll
      for (int mt = 0; mt < 4; ++mt) h1[mt] = mx(f1[(mt * 21 + kb) * 64 + l], xb[kb], h1[mt]);
    uint32_t bits = 0;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int m = 16 * mt + 4 * g + i;
        const float t = m < NP1 ? h1[mt][i] + sv[H2::B1 + m] : 0.f;
        if (t > 0.f) bits |= 1u << (4 * mt + i);
        h1[mt][i] = fmaxf(t, 0.f);
      }
    // (2) a2 = W2 h1 + b2; y = W3 ReLU(a2) + b3
    floatx4_t a2[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) a2[mt] = floatx4_t{0.f, 0.f, 0.f, 0.f};
    const float* f2g = lds_after(f2, h1[3][3]);
#pragma unroll
    for (int kb = 0; kb < 16; ++kb)
#pragma unroll
      for (int mt = 0; mt < 2; ++mt)
        a2[mt] = mx(f2g[(mt * 16 + kb) * 64 + l], h1[kb >> 2][kb & 3], a2[mt]);
    float ys = 0.f;
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int m = 16 * mt + 4 * g + i;
        if (m < NP2) {
          const float t = a2[mt][i] + sv[H2::B2 + m];
          if (t > 0.f) bits |= 1u << (16 + 4 * mt + i);
          ys = fmaf(sv[H2::W3 + m], fmaxf(t, 0.f), ys);
        }
      }
    ys += __shfl_xor(ys, 16, 64);
    ys += __shfl_xor(ys, 32, 64);
    const float y = ys + sv[H2::B3];
    const float a = (float)prm[item * NPRM + 6];
    if (g == 0) aux[v] = 1.f / (1.f + expf(-a * y));
    sgn[v * 4 + g] = bits;
  }
}

// Position network, adjoint: from Mbar (mbar), pos and m (aux, aux + total) and the stored
// ReLU signs, u = W1^T ([a1 > 0] W2^T ([a2 > 0] W3 ybar)) with ybar = Mbar m a pos (1 - pos),
// written to U [B n^3 / 16][81][16] (per 16-voxel group, feature-major: one 5 KB block).
__global__ __launch_bounds__(64 * MX_WAVES) void halo2_mx_bwd_kernel(
    int log_n, size_t groups, size_t total, const float* __restrict__ w,
    const double* __restrict__ prm, const float* __restrict__ mbar,
    const float* __restrict__ aux, const uint32_t* __restrict__ sgn, float* __restrict__ U) {
  constexpr int NFRAG = H2::SIZE - H2::F3;
  __shared__ __attribute__((aligned(16))) float sf[NFRAG];
  __shared__ float sw3[32];  // W3, read per lane group
  for (int i = threadIdx.x; i < NFRAG / 4; i += 64 * MX_WAVES)
    reinterpret_cast<float4*>(sf)[i] = reinterpret_cast<const float4*>(w + H2::F3)[i];
  if (threadIdx.x < 32) sw3[threadIdx.x] = w[H2::W3 + threadIdx.x];
  __syncthreads();
  const float* f3 = sf;
  const float* f4 = sf + (H2::F4 - H2::F3);
  const int l = threadIdx.x & 63, g = l >> 4, n = l & 15;
  const size_t stride = (size_t)gridDim.x * MX_WAVES;
  for (size_t G = (size_t)xcd_block(blockIdx.x, gridDim.x) * MX_WAVES + (threadIdx.x >> 6);
       G < groups; G += stride) {
    const size_t v = G * 16 + n;
    const size_t item = v >> (3 * log_n);
    const uint32_t bits = sgn[v * 4 + g];
    const float pos = aux[v];
    const float a = (float)prm[item * NPRM + 6];
    const float yb = mbar[v] * aux[total + v] * a * pos * (1.f - pos);
    // (3) a1bar = W2^T a2bar, masked by the layer-1 ReLU
    floatx4_t a2b[2];
#pragma unroll
    for (int mt = 0; mt < 2; ++mt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int m = 16 * mt + 4 * g + i;
        a2b[mt][i] = (m < NP2 && ((bits >> (16 + 4 * mt + i)) & 1)) ? sw3[m] * yb : 0.f;
      }
    floatx4_t a1b[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) a1b[mt] = floatx4_t{0.f, 0.f, 0.f, 0.f};
    const float* f3g = lds_after(f3, a2b[1][3]);
#pragma unroll
    for (int kb = 0; kb < 8; ++kb)
#pragma unroll
      for (int mt = 0; mt < 4; ++mt)
        a1b[mt] = mx(f3g[(mt * 8 + kb) * 64 + l], a2b[kb >> 2][kb & 3], a1b[mt]);
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
      for (int i = 0; i < 4; ++i) a1b[mt][i] = ((bits >> (4 * mt + i)) & 1) ? a1b[mt][i] : 0.f;
    // (4) u = W1^T a1bar, written per feature
    floatx4_t u[6];
#pragma unroll
    for (int mt = 0; mt < 6; ++mt) u[mt] = floatx4_t{0.f, 0.f, 0.f, 0.f};
    const float* f4g = lds_after(f4, a1b[3][3]);
#pragma unroll
    for (int kb = 0; kb < 16; ++kb)
#pragma unroll
      for (int mt = 0; mt < 6; ++mt)
        u[mt] = mx(f4g[(mt * 16 + kb) * 64 + l], a1b[kb >> 2][kb & 3], u[mt]);
    float* uo = U + G * NF * 16 + n;  // [group][feature][16]: one 5 KB block per group
#pragma unroll
    for (int mt = 0; mt < 6; ++mt)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int f = 16 * mt + 4 * g + i;
        if (f < NF) uo[f * 16] = u[mt][i];
      }
  }
}

}  // namespace

void launch_halo2_prepare(const float* nnp, const float* nnm, float* w, hipStream_t s) {
  halo2_prepare_kernel<<<(H2::SIZE + TB - 1) / TB, TB, 0, s>>>(nnp, nnm, w);
}

template <auto Kernel>
int mx_grid(size_t total) {
  const size_t groups = total / 16, waves = (groups + MX_WAVES - 1) / MX_WAVES;
  const int res = resident_grid<Kernel, 64 * MX_WAVES>();
  return (int)(waves < (size_t)res ? waves : (size_t)res);
}

void launch_halo2_fwd(const float* d0, const float* d1, const float* d2, int log_n, size_t total,
                      const float* w, const double* prm, float* aux, uint32_t* sgn, float* mass,
                      hipStream_t s) {
  halo2_mx_fwd_kernel<<<mx_grid<halo2_mx_fwd_kernel>(total), 64 * MX_WAVES, 0, s>>>(
      d0, d1, d2, log_n, total / 16, w, prm, aux, sgn);
  halo2_nnm_kernel<false><<<(unsigned)((total + TB - 1) / TB), TB, 0, s>>>(
      d0, d1, d2, total, w, aux, nullptr, aux + total, mass, nullptr, nullptr, nullptr);
}

void launch_halo2_bwd(const float* d0, const float* d1, const float* d2, int log_n, size_t total,
                      const float* w, const double* prm, const float* mbar, const float* aux,
                      const uint32_t* sgn, float* U, float* g0, float* g12, float* g2,
                      hipStream_t s) {
  halo2_mx_bwd_kernel<<<mx_grid<halo2_mx_bwd_kernel>(total), 64 * MX_WAVES, 0, s>>>(
      log_n, total / 16, total, w, prm, mbar, aux, sgn, U);
  halo2_nnm_kernel<true><<<(unsigned)((total + TB - 1) / TB), TB, 0, s>>>(
      d0, d1, d2, total, w, aux, mbar, nullptr, nullptr, g0, g12, g2);
}

void launch_halo2_stencil_adj(const float* U, int log_n, size_t total, float* g0, float* g12,
                              float* g2, hipStream_t s) {
  halo2_stencil_adj_kernel<<<(unsigned)((total + TB - 1) / TB), TB, 0, s>>>(U, log_n, total, g0,
                                                                            g12, g2);
}

}  // namespace pmr
