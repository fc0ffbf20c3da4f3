// Halo-mass model and likelihood on the output mesh (Sec. 2.1, Sec. 2.2, Sec. 5.1).
//
// Per voxel: features f = (delta_0, delta_R1, delta_R1 - delta_R2); a 3 -> H -> H -> 1
// network with ReLU hidden layers and a softplus on the output gives the mass M.
// Likelihood: x = log(M_R + M0), residual r = (mu + x - x_data) / (2 sigma_N); the
// residual is Gaussian-smoothed on R_sm (the anneal) and squared. Sums are reduced in
// FP64 with a fixed tree, so the loss is bitwise reproducible.
//
// Loss parameters live in device memory, [B][6] doubles:
//   (M0, mu, sigma_N, R_mass, R_sm, prior_weight).
#include "pmr_internal.h"

namespace pmr {
namespace {

constexpr int TB = 256;

__device__ __forceinline__ float softplus_f(float y) {
  return fmaxf(y, 0.f) + log1pf(expf(-fabsf(y)));
}
__device__ __forceinline__ float sigmoid_f(float y) { return 1.f / (1.f + expf(-y)); }

// Weight block layout (floats): W1[H][3], b1[H], W2[H][H], b2[H], W3[H], b3[1].
template <int H>
struct WOff {
  static constexpr int W1 = 0, B1 = 3 * H, W2 = 4 * H, B2 = 4 * H + H * H, W3 = 5 * H + H * H,
                       B3 = 6 * H + H * H, SIZE = 6 * H + H * H + 1;
};

template <int H>
__device__ __forceinline__ void load_weights(float* sw, const float* __restrict__ w) {
  for (int i = threadIdx.x; i < WOff<H>::SIZE; i += TB) sw[i] = w[i];
  __syncthreads();
}

// M = softplus(W3 relu(W2 relu(W1 f + b1) + b2) + b3), FP32.
template <int H>
__global__ __launch_bounds__(TB) void mlp_fwd_kernel(const float* __restrict__ d0,
                                                     const float* __restrict__ d1,
                                                     const float* __restrict__ d2, size_t n,
                                                     const float* __restrict__ w,
                                                     float* __restrict__ mass) {
  using O = WOff<H>;
  __shared__ float sw[O::SIZE];
  load_weights<H>(sw, w);
  const size_t v = (size_t)blockIdx.x * TB + threadIdx.x;
  if (v >= n) return;
  const float f0 = d0[v], f1 = d1[v], f2 = d1[v] - d2[v];
  float h1[H];
#pragma unroll
  for (int j = 0; j < H; ++j)
    h1[j] = fmaxf(sw[O::W1 + 3 * j] * f0 + sw[O::W1 + 3 * j + 1] * f1 + sw[O::W1 + 3 * j + 2] * f2 +
                      sw[O::B1 + j],
                  0.f);
  float y = sw[O::B3];
#pragma unroll 4
  for (int j = 0; j < H; ++j) {
    float a = sw[O::B2 + j];
#pragma unroll
    for (int i = 0; i < H; ++i) a += sw[O::W2 + j * H + i] * h1[i];
    y += sw[O::W3 + j] * fmaxf(a, 0.f);
  }
  mass[v] = softplus_f(y);
}

// Input gradient with weights frozen (recomputing the forward pass):
//   ybar = Mbar sigmoid(y); a2bar = ybar W3 [a2 > 0]; a1bar = (W2^T a2bar) [a1 > 0];
//   fbar = W1^T a1bar. Writes fbar0, fbar1 + fbar2 and fbar2 (the features' adjoint needs
//   G_R1 (fbar1 + fbar2) - G_R2 fbar2).
template <int H>
__global__ __launch_bounds__(TB) void mlp_bwd_kernel(const float* __restrict__ d0,
                                                     const float* __restrict__ d1,
                                                     const float* __restrict__ d2, size_t n,
                                                     const float* __restrict__ w,
                                                     const float* __restrict__ mbar,
                                                     float* __restrict__ g0, float* __restrict__ g12,
                                                     float* __restrict__ g2) {
  using O = WOff<H>;
  __shared__ float sw[O::SIZE];
  load_weights<H>(sw, w);
  const size_t v = (size_t)blockIdx.x * TB + threadIdx.x;
  if (v >= n) return;
  const float f0 = d0[v], f1 = d1[v], f2 = d1[v] - d2[v];
  float a1[H], a2[H];
#pragma unroll
  for (int j = 0; j < H; ++j)
    a1[j] = sw[O::W1 + 3 * j] * f0 + sw[O::W1 + 3 * j + 1] * f1 + sw[O::W1 + 3 * j + 2] * f2 +
            sw[O::B1 + j];
  float y = sw[O::B3];
#pragma unroll 4
  for (int j = 0; j < H; ++j) {
    float a = sw[O::B2 + j];
#pragma unroll
    for (int i = 0; i < H; ++i) a += sw[O::W2 + j * H + i] * fmaxf(a1[i], 0.f);
    a2[j] = a;
    y += sw[O::W3 + j] * fmaxf(a, 0.f);
  }
  const float yb = mbar[v] * sigmoid_f(y);
#pragma unroll
  for (int j = 0; j < H; ++j) a2[j] = a2[j] > 0.f ? yb * sw[O::W3 + j] : 0.f;
  float fb0 = 0.f, fb1 = 0.f, fb2 = 0.f;
#pragma unroll 4
  for (int i = 0; i < H; ++i) {
    float hb = 0.f;
#pragma unroll
    for (int j = 0; j < H; ++j) hb += sw[O::W2 + j * H + i] * a2[j];
    if (a1[i] > 0.f) {
      fb0 += sw[O::W1 + 3 * i] * hb;
      fb1 += sw[O::W1 + 3 * i + 1] * hb;
      fb2 += sw[O::W1 + 3 * i + 2] * hb;
    }
  }
  g0[v] = fb0;
  g12[v] = fb1 + fb2;
  g2[v] = fb2;
}

// ---------------------------------------------------------------- matrix-core network
// The H x H layer runs on the matrix cores, in one of two precisions:
//   BF16: v_mfma_f32_16x16x32_bf16 (BF16 inputs, FP32 accumulation) - the mixed path;
//   FP32: v_mfma_f32_16x16x4_f32 (FP32 inputs and accumulation) - the FP32 path.
// The 3 -> H and H -> 1 layers, biases, activations and the softplus stay FP32 on the vector
// units. Operand layouts (lane l, i = 0..3), with KS the instruction's k extent and
// J = KS / 4 consecutive k per lane:
//   A[m][k]: m = l % 16, k = J (l / 16) + j      B[k][n]: n = l % 16, k = J (l / 16) + j
//   C[m][n]: n = l % 16, m = 4 (l / 16) + i
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float floatx4_t __attribute__((ext_vector_type(4)));

struct MxBF16 {
  static constexpr int KS = 32, J = 8;
  typedef bf16x8_t frag;
  typedef __bf16 elem;
  __device__ static floatx4_t mma(frag a, frag b, floatx4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  __device__ static void set(frag& f, int j, float v) { f[j] = (__bf16)v; }
  __device__ static elem cvt(float v) { return (__bf16)v; }
};

struct MxF32 {
  static constexpr int KS = 4, J = 1;
  typedef float frag;
  typedef float elem;
  __device__ static floatx4_t mma(frag a, frag b, floatx4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static void set(frag& f, int, float v) { f = v; }
  __device__ static elem cvt(float v) { return v; }
};

// Compact block of the FP32 weights the matrix-core kernels keep in LDS: W1[H][3], b1[H],
// b2[H], W3[H], b3.
template <int H>
struct SOff {
  static constexpr int W1 = 0, B1 = 3 * H, B2 = 4 * H, W3 = 5 * H, B3 = 6 * H, SIZE = 6 * H + 1;
};

template <int H>
__device__ __forceinline__ void load_small_weights(float* sw, const float* __restrict__ w) {
  using O = WOff<H>;
  for (int i = threadIdx.x; i < SOff<H>::SIZE; i += TB) {
    float v;
    if (i < 4 * H) v = w[i];  // W1 and b1 sit at the same offsets in both blocks
    else if (i < 5 * H) v = w[O::B2 + (i - 4 * H)];
    else if (i < 6 * H) v = w[O::W3 + (i - 5 * H)];
    else v = w[O::B3];
    sw[i] = v;
  }
  __syncthreads();
}

// BF16 copies of W2 (row-major [n][k]) and W2^T, placed after the FP32 block.
template <int H>
struct WBf {
  static constexpr size_t W2 = ((size_t)WOff<H>::SIZE * 4 + 15) / 16 * 16;  // byte offset
  static constexpr size_t W2T = W2 + (size_t)H * H * 2;
  static constexpr size_t BYTES = W2T + (size_t)H * H * 2;
};

template <int H>
__global__ void mlp_prepare_bf16_kernel(float* w) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= H * H) return;
  const int n = t / H, k = t % H;
  char* base = reinterpret_cast<char*>(w);
  __bf16* w2 = reinterpret_cast<__bf16*>(base + WBf<H>::W2);
  __bf16* w2t = reinterpret_cast<__bf16*>(base + WBf<H>::W2T);
  const float v = w[WOff<H>::W2 + n * H + k];
  w2[n * H + k] = (__bf16)v;
  w2t[k * H + n] = (__bf16)v;
}

__device__ __forceinline__ float group16_sum(float v) {
  v += __shfl_xor(v, 1, 64);
  v += __shfl_xor(v, 2, 64);
  v += __shfl_xor(v, 4, 64);
  v += __shfl_xor(v, 8, 64);
  return v;
}

// Row blocks of 16 voxels a wavefront processes at a time (4 VGPRs of accumulator per 16x16
// output block, so fewer blocks keep more waves resident).
constexpr int MFMA_MB = 2;

// h1 fragments (A layout) for the MB row blocks of this wave (zero past the end).
template <class P, int H, int MB>
__device__ __forceinline__ void h1_fragments(const float* sw, const float* __restrict__ d0,
                                             const float* __restrict__ d1,
                                             const float* __restrict__ d2, size_t v0, size_t n,
                                             typename P::frag (&a)[MB][H / P::KS]) {
  using S = SOff<H>;
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) {
    const size_t v = v0 + mb * 16 + (l & 15);
    float f0 = 0.f, f1 = 0.f, f2 = 0.f;
    if (v < n) {
      f0 = d0[v];
      f1 = d1[v];
      f2 = d1[v] - d2[v];
    }
#pragma unroll
    for (int kb = 0; kb < H / P::KS; ++kb) {
#pragma unroll
      for (int j = 0; j < P::J; ++j) {
        const int k = kb * P::KS + P::J * (l >> 4) + j;
        const float h = fmaxf(sw[S::W1 + 3 * k] * f0 + sw[S::W1 + 3 * k + 1] * f1 +
                                  sw[S::W1 + 3 * k + 2] * f2 + sw[S::B1 + k],
                              0.f);
        P::set(a[mb][kb], j, h);
      }
    }
  }
}

// B fragments of a row-major [n][k] matrix m with row pitch RP (B[k][n] = m[n][k]).
template <class P, int H, int RP = H>
__device__ __forceinline__ void load_b(const typename P::elem* __restrict__ m,
                                       typename P::frag (&b)[H / P::KS][H / 16]) {
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int kb = 0; kb < H / P::KS; ++kb)
#pragma unroll
    for (int nb = 0; nb < H / 16; ++nb)
      b[kb][nb] = *reinterpret_cast<const typename P::frag*>(
          m + (size_t)(nb * 16 + (l & 15)) * RP + kb * P::KS + P::J * (l >> 4));
}

template <class P, int H, int MB>
__device__ __forceinline__ void mfma_layer(const typename P::frag (&a)[MB][H / P::KS],
                                           const typename P::frag (&b)[H / P::KS][H / 16],
                                           floatx4_t (&c)[MB][H / 16]) {
#pragma unroll
  for (int mb = 0; mb < MB; ++mb)
#pragma unroll
    for (int nb = 0; nb < H / 16; ++nb) {
      floatx4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kb = 0; kb < H / P::KS; ++kb) acc = P::mma(a[mb][kb], b[kb][nb], acc);
      c[mb][nb] = acc;
    }
}

// y for the 4 rows (4 (l/16) + i) of row block mb, on every lane of the 16-lane group.
template <int H, int MB>
__device__ __forceinline__ void layer3(const float* sw, const floatx4_t (&c)[MB][H / 16], int mb,
                                       float (&y)[4]) {
  using S = SOff<H>;
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    float p = 0.f;
#pragma unroll
    for (int nb = 0; nb < H / 16; ++nb) {
      const int nn = nb * 16 + (l & 15);
      p += sw[S::W3 + nn] * fmaxf(c[mb][nb][i] + sw[S::B2 + nn], 0.f);
    }
    y[i] = group16_sum(p) + sw[S::B3];
  }
}

// W2 (row-major [n][k]) and W2^T in the element type of P: the BF16 copies after the FP32
// block, or (FP32) the block's own W2 and a transposed copy made in LDS by the caller.
template <class P, int H>
__device__ __forceinline__ const typename P::elem* w2_rows(const float* w) {
  if constexpr (sizeof(typename P::elem) == 2)
    return reinterpret_cast<const typename P::elem*>(reinterpret_cast<const char*>(w) + WBf<H>::W2);
  else
    return reinterpret_cast<const typename P::elem*>(w + WOff<H>::W2);
}

// Persistent: each wavefront walks groups of 16 MB voxels (wave, wave + all waves, ...) with
// the small FP32 weights in LDS and the W2 fragments in registers, loaded once.
template <class P, int H>
__global__ __launch_bounds__(TB) void mlp_fwd_mx_kernel(const float* __restrict__ d0,
                                                        const float* __restrict__ d1,
                                                        const float* __restrict__ d2, size_t n,
                                                        const float* __restrict__ w,
                                                        float* __restrict__ mass) {
  using S = SOff<H>;
  constexpr int MB = MFMA_MB, GV = 16 * MB;  // voxels per group
  __shared__ float sw[S::SIZE];
  load_small_weights<H>(sw, w);
  const int l = threadIdx.x & 63;
  typename P::frag b[H / P::KS][H / 16];
  load_b<P, H>(w2_rows<P, H>(w), b);
  const size_t groups = (n + GV - 1) / GV;
  const size_t nwaves = (size_t)gridDim.x * (TB / 64);
  for (size_t g = (size_t)blockIdx.x * (TB / 64) + (threadIdx.x >> 6); g < groups; g += nwaves) {
    const size_t v0 = g * GV;
    typename P::frag a[MB][H / P::KS];
    floatx4_t c[MB][H / 16];
    h1_fragments<P, H, MB>(sw, d0, d1, d2, v0, n, a);
    mfma_layer<P, H, MB>(a, b, c);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      float y[4];
      layer3<H, MB>(sw, c, mb, y);
      const int i = l & 15;
      if (i < 4) {
        const size_t v = v0 + mb * 16 + 4 * (l >> 4) + i;
        const float yi = i == 0 ? y[0] : i == 1 ? y[1] : i == 2 ? y[2] : y[3];
        if (v < n) mass[v] = softplus_f(yi);
      }
    }
  }
}

// Input gradient (weights frozen, forward recomputed), as mlp_bwd_kernel, with both H x H
// products (W2 h1 and W2^T a2bar) on the matrix cores.
template <class P, int H>
__global__ __launch_bounds__(TB) void mlp_bwd_mx_kernel(const float* __restrict__ d0,
                                                        const float* __restrict__ d1,
                                                        const float* __restrict__ d2, size_t n,
                                                        const float* __restrict__ w,
                                                        const float* __restrict__ mbar,
                                                        float* __restrict__ g0,
                                                        float* __restrict__ g12,
                                                        float* __restrict__ g2) {
  using S = SOff<H>;
  using E = typename P::elem;
  constexpr int MB = MFMA_MB, GV = 16 * MB;  // voxels per group
  __shared__ float sw[S::SIZE];
  // Row pitch RP: rows of the LDS copies are padded so that the 16 rows a fragment read
  // touches fall on distinct banks. 16-byte aligned: BF16 fragments are 16-byte vectors.
  constexpr int RP = H + (sizeof(E) == 2 ? 8 : 1);
  __shared__ __attribute__((aligned(16))) E wm[2 * H * RP];  // W2 and W2^T, row-major
  __shared__ __attribute__((aligned(16))) E tile[TB / 64][GV * RP];
  {
    const E* w2 = w2_rows<P, H>(w);
    for (int i = threadIdx.x; i < H * H; i += TB) {
      const int r = i / H, c = i % H;
      const E v = w2[i];
      wm[r * RP + c] = v;
      wm[H * RP + c * RP + r] = v;
    }
  }
  load_small_weights<H>(sw, w);  // ends with a barrier
  const int l = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  E* T = tile[wv];
  const size_t groups = (n + GV - 1) / GV;
  const size_t nwaves = (size_t)gridDim.x * (TB / 64);
  for (size_t g = (size_t)blockIdx.x * (TB / 64) + wv; g < groups; g += nwaves) {
    const size_t v0 = g * GV;
    floatx4_t c[MB][H / 16];
    {
      typename P::frag a[MB][H / P::KS];
      typename P::frag b[H / P::KS][H / 16];
      h1_fragments<P, H, MB>(sw, d0, d1, d2, v0, n, a);
      load_b<P, H, RP>(wm, b);
      mfma_layer<P, H, MB>(a, b, c);
    }
    // a2bar = ybar W3 [a2 > 0], stored as a GV x H tile for the transposed read
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      float y[4];
      layer3<H, MB>(sw, c, mb, y);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = mb * 16 + 4 * (l >> 4) + i;
        const size_t v = v0 + r;
        const float yb = v < n ? mbar[v] * sigmoid_f(y[i]) : 0.f;
#pragma unroll
        for (int nb = 0; nb < H / 16; ++nb) {
          const int nn = nb * 16 + (l & 15);
          const float a2 = c[mb][nb][i] + sw[S::B2 + nn];
          T[r * RP + nn] = P::cvt(a2 > 0.f ? yb * sw[S::W3 + nn] : 0.f);
        }
      }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_s_waitcnt(0xc07f);
    // h1bar = a2bar W2 on the matrix cores (B = W2 read as W2^T rows)
    {
      typename P::frag a[MB][H / P::KS];
      typename P::frag b[H / P::KS][H / 16];
#pragma unroll
      for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int kb = 0; kb < H / P::KS; ++kb)
          a[mb][kb] = *reinterpret_cast<const typename P::frag*>(
              T + (mb * 16 + (l & 15)) * RP + kb * P::KS + P::J * (l >> 4));
      load_b<P, H, RP>(wm + H * RP, b);
      mfma_layer<P, H, MB>(a, b, c);
    }
    // the tile is rewritten by the next group: its reads above must have completed
    __builtin_amdgcn_s_waitcnt(0xc07f);
    __builtin_amdgcn_wave_barrier();
    // a1bar = h1bar [a1 > 0]; fbar = W1^T a1bar (rows of the C layout)
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const size_t v = v0 + mb * 16 + 4 * (l >> 4) + i;
        float f0 = 0.f, f1 = 0.f, f2 = 0.f;
        if (v < n) {
          f0 = d0[v];
          f1 = d1[v];
          f2 = d1[v] - d2[v];
        }
        float p0 = 0.f, p1 = 0.f, p2 = 0.f;
#pragma unroll
        for (int nb = 0; nb < H / 16; ++nb) {
          const int k = nb * 16 + (l & 15);
          const float a1 = sw[S::W1 + 3 * k] * f0 + sw[S::W1 + 3 * k + 1] * f1 +
                           sw[S::W1 + 3 * k + 2] * f2 + sw[S::B1 + k];
          const float hb = a1 > 0.f ? c[mb][nb][i] : 0.f;
          p0 += sw[S::W1 + 3 * k] * hb;
          p1 += sw[S::W1 + 3 * k + 1] * hb;
          p2 += sw[S::W1 + 3 * k + 2] * hb;
        }
        p0 = group16_sum(p0);
        p1 = group16_sum(p1);
        p2 = group16_sum(p2);
        if ((l & 15) == i && v < n) {
          g0[v] = p0;
          g12[v] = p1 + p2;
          g2[v] = p2;
        }
      }
    }
  }
}

// x_data = log(MtR + M0)
__global__ void target_x_kernel(const float* __restrict__ mtr, size_t per_item, int batch,
                                const double* __restrict__ prm, float* __restrict__ xd) {
  const size_t v = (size_t)blockIdx.x * TB + threadIdx.x;
  if (v >= per_item * batch) return;
  const int b = (int)(v / per_item);
  xd[v] = logf(mtr[v] + (float)prm[b * 6 + 0]);
}

// r = (mu + log(MR + M0) - x_data) / (2 sigma_N)
__global__ void residual_kernel(const float* __restrict__ mr, const float* __restrict__ xd,
                                size_t per_item, int batch, const double* __restrict__ prm,
                                float* __restrict__ r) {
  const size_t v = (size_t)blockIdx.x * TB + threadIdx.x;
  if (v >= per_item * batch) return;
  const int b = (int)(v / per_item);
  const float M0 = (float)prm[b * 6 + 0], mu = (float)prm[b * 6 + 1];
  const float inv2s = (float)(0.5 / prm[b * 6 + 2]);
  r[v] = (mu + logf(mr[v] + M0) - xd[v]) * inv2s;
}

// MRbar = rbar / (2 sigma_N (MR + M0))
__global__ void mrbar_kernel(const float* __restrict__ rbar, const float* __restrict__ mr,
                             size_t per_item, int batch, const double* __restrict__ prm,
                             float* __restrict__ out) {
  const size_t v = (size_t)blockIdx.x * TB + threadIdx.x;
  if (v >= per_item * batch) return;
  const int b = (int)(v / per_item);
  const float M0 = (float)prm[b * 6 + 0];
  const float inv2s = (float)(0.5 / prm[b * 6 + 2]);
  out[v] = rbar[v] * inv2s / (mr[v] + M0);
}

// density-L2 adjoint: dbar = 2 loss_bar (delta - target) (+ extra)
__global__ void l2_adj_kernel(const float* __restrict__ d, const float* __restrict__ t,
                              size_t per_item, int batch, const double* __restrict__ loss_bar,
                              const float* __restrict__ extra, float* __restrict__ out) {
  const size_t v = (size_t)blockIdx.x * TB + threadIdx.x;
  if (v >= per_item * batch) return;
  const int b = (int)(v / per_item);
  float g = 2.f * (float)loss_bar[b] * (d[v] - t[v]);
  if (extra) g += extra[v];
  out[v] = g;
}

// ---------------------------------------------------------------- FP64 reductions
__device__ __forceinline__ double block_sum_fixed(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
#pragma unroll
  for (int s = TB / 2; s > 0; s >>= 1) {
    if (t < s) sh[t] += sh[t + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

constexpr int RED_ITEMS = 16;
constexpr int RED_TILE = TB * RED_ITEMS;

// partial[b * nblk + blk] = sum over the tile of (a - c)^2 (c nullable), FP64 accumulation.
__global__ __launch_bounds__(TB) void sumsq_partial_kernel(const float* __restrict__ a,
                                                           const float* __restrict__ c,
                                                           size_t per_item, int nblk,
                                                           double* __restrict__ partial) {
  __shared__ double sh[TB];
  const int b = blockIdx.y;
  const size_t base = (size_t)b * per_item + (size_t)blockIdx.x * RED_TILE;
  const size_t lim = (size_t)b * per_item + per_item;
  double s = 0.0;
  for (int i = 0; i < RED_ITEMS; ++i) {
    const size_t j = base + (size_t)i * TB + threadIdx.x;
    if (j < lim) {
      const double d = c ? (double)a[j] - (double)c[j] : (double)a[j];
      s += d * d;
    }
  }
  const double tot = block_sum_fixed(s, sh);
  if (threadIdx.x == 0) partial[(size_t)b * nblk + blockIdx.x] = tot;
}

// out[b] = sum_k partial[b][k] in a fixed order (one block per item)
__global__ __launch_bounds__(TB) void sum_partials_kernel(const double* __restrict__ partial,
                                                          int nblk, double* __restrict__ out) {
  __shared__ double sh[TB];
  const int b = blockIdx.x;
  double s = 0.0;
  for (int k = threadIdx.x; k < nblk; k += TB) s += partial[(size_t)b * nblk + k];
  const double tot = block_sum_fixed(s, sh);
  if (threadIdx.x == 0) out[b] = tot;
}

// loss_out[b] = (prior_weight * prior + data, prior, data)
__global__ void finalize_loss_kernel(const double* __restrict__ prior, const double* __restrict__ data,
                                     const double* __restrict__ prm, int batch,
                                     double* __restrict__ loss_out) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  loss_out[3 * b + 0] = prm[b * 6 + 5] * prior[b] + data[b];
  loss_out[3 * b + 1] = prior[b];
  loss_out[3 * b + 2] = data[b];
}

// ---------------------------------------------------------------- modes
// P s on the stored half spectrum: on kz in {0, n/2} average with conj of the (-i, -j)
// partner; zero k = 0. Also the prior partial sums 0.5 * w * |P s|^2 / S.
__global__ __launch_bounds__(TB) void project_prior_kernel(const float2* __restrict__ s, int n,
                                                           const float* __restrict__ inv_var,
                                                           float2* __restrict__ ps, int nblk,
                                                           double* __restrict__ partial) {
  __shared__ double sh[TB];
  const int nh = n / 2 + 1;
  const size_t per = (size_t)n * n * nh;
  const int b = blockIdx.y;
  const float2* sb = s + b * per;
  double acc = 0.0;
  for (int i = 0; i < RED_ITEMS; ++i) {
    const size_t e = (size_t)blockIdx.x * RED_TILE + (size_t)i * TB + threadIdx.x;
    if (e >= per) continue;
    const int kz = (int)(e % nh);
    const int iy = (int)((e / nh) % n);
    const int ix = (int)(e / ((size_t)nh * n));
    float2 v = sb[e];
    double w = 2.0;
    if (kz == 0 || kz == n / 2) {
      const int jx = (n - ix) & (n - 1), jy = (n - iy) & (n - 1);
      const float2 q = sb[((size_t)jx * n + jy) * nh + kz];
      v = make_float2(0.5f * (v.x + q.x), 0.5f * (v.y - q.y));
      w = 1.0;
    }
    if (e == 0) v = make_float2(0.f, 0.f);
    ps[b * per + e] = v;
    acc += 0.5 * w * ((double)v.x * v.x + (double)v.y * v.y) * (double)inv_var[e];
  }
  const double tot = block_sum_fixed(acc, sh);
  if (threadIdx.x == 0) partial[(size_t)b * nblk + blockIdx.x] = tot;
}

template <int H>
void mlp_fwd_t(const float* d0, const float* d1, const float* d2, size_t n, const float* w,
               float* mass, hipStream_t s) {
  mlp_fwd_kernel<H><<<(unsigned)((n + TB - 1) / TB), TB, 0, s>>>(d0, d1, d2, n, w, mass);
}
template <int H>
void mlp_bwd_t(const float* d0, const float* d1, const float* d2, size_t n, const float* w,
               const float* mbar, float* g0, float* g12, float* g2, hipStream_t s) {
  mlp_bwd_kernel<H><<<(unsigned)((n + TB - 1) / TB), TB, 0, s>>>(d0, d1, d2, n, w, mbar, g0, g12,
                                                                 g2);
}

}  // namespace

size_t mlp_weight_floats(int H) {
  // FP32 block, then BF16 W2 and W2^T (16-byte aligned)
  return ((size_t)6 * H + (size_t)H * H + 1 + 3) / 4 * 4 + (size_t)H * H + 4;
}

int launch_mlp_prepare_bf16(int H, float* w, hipStream_t s) {
  switch (H) {
    case 32: mlp_prepare_bf16_kernel<32><<<(32 * 32 + 255) / 256, 256, 0, s>>>(w); return 0;
    case 64: mlp_prepare_bf16_kernel<64><<<(64 * 64 + 255) / 256, 256, 0, s>>>(w); return 0;
    default: return -1;
  }
}

// Workgroups of the persistent matrix-core kernels: the resident number, fewer when the
// mesh is small.
template <auto Kernel>
static unsigned mx_blocks(size_t n) {
  const size_t need = (n + TB - 1) / TB;
  const size_t res = (size_t)resident_grid<Kernel, TB>();
  return (unsigned)(need < res ? need : res);
}

template <class P, int H>
static void mlp_fwd_mx_t(const float* d0, const float* d1, const float* d2, size_t n,
                         const float* w, float* mass, hipStream_t s) {
  constexpr auto k = mlp_fwd_mx_kernel<P, H>;
  k<<<mx_blocks<k>(n), TB, 0, s>>>(d0, d1, d2, n, w, mass);
}
template <class P, int H>
static void mlp_bwd_mx_t(const float* d0, const float* d1, const float* d2, size_t n,
                         const float* w, const float* mbar, float* g0, float* g12, float* g2,
                         hipStream_t s) {
  constexpr auto k = mlp_bwd_mx_kernel<P, H>;
  k<<<mx_blocks<k>(n), TB, 0, s>>>(d0, d1, d2, n, w, mbar, g0, g12, g2);
}

int launch_mlp_fwd_mfma(int H, const float* d0, const float* d1, const float* d2, size_t n,
                        const float* w, float* mass, hipStream_t s) {
  switch (H) {
    case 32: mlp_fwd_mx_t<MxBF16, 32>(d0, d1, d2, n, w, mass, s); return 0;
    case 64: mlp_fwd_mx_t<MxBF16, 64>(d0, d1, d2, n, w, mass, s); return 0;
    default: return -1;
  }
}

int launch_mlp_bwd_mfma(int H, const float* d0, const float* d1, const float* d2, size_t n,
                        const float* w, const float* mbar, float* g0, float* g12, float* g2,
                        hipStream_t s) {
  switch (H) {
    case 32: mlp_bwd_mx_t<MxBF16, 32>(d0, d1, d2, n, w, mbar, g0, g12, g2, s); return 0;
    case 64: mlp_bwd_mx_t<MxBF16, 64>(d0, d1, d2, n, w, mbar, g0, g12, g2, s); return 0;
    default: return -1;
  }
}

// FP32 network: H x H layer on the FP32 matrix cores where H is a multiple of 16, else one
// thread per voxel on the vector units.
int launch_mlp_fwd(int H, const float* d0, const float* d1, const float* d2, size_t n,
                   const float* w, float* mass, hipStream_t s) {
  switch (H) {
    case 8: mlp_fwd_t<8>(d0, d1, d2, n, w, mass, s); return 0;
    case 16: mlp_fwd_mx_t<MxF32, 16>(d0, d1, d2, n, w, mass, s); return 0;
    case 32: mlp_fwd_mx_t<MxF32, 32>(d0, d1, d2, n, w, mass, s); return 0;
    case 64: mlp_fwd_mx_t<MxF32, 64>(d0, d1, d2, n, w, mass, s); return 0;
    default: return -1;
  }
}

int launch_mlp_bwd(int H, const float* d0, const float* d1, const float* d2, size_t n,
                   const float* w, const float* mbar, float* g0, float* g12, float* g2,
                   hipStream_t s) {
  switch (H) {
    case 8: mlp_bwd_t<8>(d0, d1, d2, n, w, mbar, g0, g12, g2, s); return 0;
    case 16: mlp_bwd_mx_t<MxF32, 16>(d0, d1, d2, n, w, mbar, g0, g12, g2, s); return 0;
    case 32: mlp_bwd_mx_t<MxF32, 32>(d0, d1, d2, n, w, mbar, g0, g12, g2, s); return 0;
    case 64: mlp_bwd_mx_t<MxF32, 64>(d0, d1, d2, n, w, mbar, g0, g12, g2, s); return 0;
    default: return -1;
  }
}

static unsigned grid1(size_t n) { return (unsigned)((n + TB - 1) / TB); }

void launch_target_x(const float* mtr, size_t per_item, int batch, const double* prm, float* xd,
                     hipStream_t s) {
  target_x_kernel<<<grid1(per_item * batch), TB, 0, s>>>(mtr, per_item, batch, prm, xd);
}
void launch_residual(const float* mr, const float* xd, size_t per_item, int batch,
                     const double* prm, float* r, hipStream_t s) {
  residual_kernel<<<grid1(per_item * batch), TB, 0, s>>>(mr, xd, per_item, batch, prm, r);
}
void launch_mrbar(const float* rbar, const float* mr, size_t per_item, int batch,
                  const double* prm, float* out, hipStream_t s) {
  mrbar_kernel<<<grid1(per_item * batch), TB, 0, s>>>(rbar, mr, per_item, batch, prm, out);
}
void launch_l2_adj(const float* d, const float* t, size_t per_item, int batch,
                   const double* loss_bar, const float* extra, float* out, hipStream_t s) {
  l2_adj_kernel<<<grid1(per_item * batch), TB, 0, s>>>(d, t, per_item, batch, loss_bar, extra, out);
}

int reduce_blocks(size_t per_item) { return (int)((per_item + RED_TILE - 1) / RED_TILE); }

// out[b] = sum over item b of (a - c)^2, deterministic.
void launch_sumsq(const float* a, const float* c, size_t per_item, int batch, double* partial,
                  double* out, hipStream_t s) {
  const int nblk = reduce_blocks(per_item);
  sumsq_partial_kernel<<<dim3(nblk, batch), TB, 0, s>>>(a, c, per_item, nblk, partial);
  sum_partials_kernel<<<batch, TB, 0, s>>>(partial, nblk, out);
}

void launch_project_prior(const float2* modes, int n, int batch, const float* inv_var, float2* ps,
                          double* partial, double* prior_out, hipStream_t s) {
  const size_t per = (size_t)n * n * (n / 2 + 1);
  const int nblk = reduce_blocks(per);
  project_prior_kernel<<<dim3(nblk, batch), TB, 0, s>>>(modes, n, inv_var, ps, nblk, partial);
  sum_partials_kernel<<<batch, TB, 0, s>>>(partial, nblk, prior_out);
}

void launch_finalize_loss(const double* prior, const double* data, const double* prm, int batch,
                          double* loss_out, hipStream_t s) {
  finalize_loss_kernel<<<(batch + 63) / 64, 64, 0, s>>>(prior, data, prm, batch, loss_out);
}

}  // namespace pmr
