// Halo-mass model and likelihood on the output mesh (Sec. 2.1, Sec. 2.2, Sec. 5.1).
//
// Per voxel: features f = (delta_0, delta_R1, delta_R1 - delta_R2); a 3 -> H -> H -> 1
// network with ReLU hidden layers and a softplus on the output gives the mass M.
// Likelihood: x = log(M_R + M0), residual r = (mu + x - x_data) / (2 sigma_N); the
// residual is Gaussian-smoothed on R_sm (the anneal) and squared. Sums are reduced in
// FP64 with a fixed tree, so the loss is bitwise reproducible.
//
// Loss parameters live in device memory, [B][NPRM] doubles:
//   (M0, mu, sigma_N, R_mass, R_sm, prior_weight, logistic_a).
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

// Compact block of the FP32 weights the matrix-core kernels keep in LDS, per neuron:
// (W1[k][0..2], b1[k]) as one float4 at 4 k, then (b2[u], W3[u]) as one float2 at 4 H + 2 u,
// then b3.
template <int H>
struct SOff {
  static constexpr int L1 = 0, L2 = 4 * H, B3 = 6 * H, SIZE = 6 * H + 1;
};

template <int H>
__device__ __forceinline__ void load_small_weights(float* sw, const float* __restrict__ w) {
  using O = WOff<H>;
  for (int i = threadIdx.x; i < SOff<H>::SIZE; i += TB) {
    float v;
    if (i < 4 * H) {
      const int k = i >> 2, e = i & 3;
      v = e < 3 ? w[O::W1 + 3 * k + e] : w[O::B1 + k];
    } else if (i < 6 * H) {
      const int u = (i - 4 * H) >> 1;
      v = (i & 1) ? w[O::W3 + u] : w[O::B2 + u];
    } else {
      v = w[O::B3];
    }
    sw[i] = v;
  }
  __syncthreads();
}

template <int H>
__device__ __forceinline__ float4 l1_row(const float* sw, int k) {
  return *reinterpret_cast<const float4*>(sw + SOff<H>::L1 + 4 * k);
}
template <int H>
__device__ __forceinline__ float2 l2_row(const float* sw, int u) {
  return *reinterpret_cast<const float2*>(sw + SOff<H>::L2 + 2 * u);
}

// Where the register budget is tight (the BF16 network, whose vector work bounds it, and
// H = 64), the per-neuron weights are read from LDS where they are used rather than held in
// registers across the group loop (an opaque zero offset keeps the compiler from hoisting
// them), so that more waves stay resident. The FP32 network at H <= 32 is bound by its
// matrix-core work and keeps them in registers.
template <class P, int H>
__device__ __forceinline__ const float* lds_fence(const float* sw) {
  if constexpr (sizeof(typename P::elem) == 2 || H >= 64) {
    int z = 0;
    asm volatile("" : "+v"(z));
    return sw + z;
  } else {
    return sw;
  }
}

// BF16 copy of W2 (row-major [n][k]), placed after the FP32 block (16-byte aligned); the
// matrix-core kernels read both W2 and W2^T fragments from it.
template <int H>
struct WBf {
  static constexpr size_t W2 = ((size_t)WOff<H>::SIZE * 4 + 15) / 16 * 16;  // byte offset
  static constexpr size_t BYTES = W2 + (size_t)H * H * 2;
};

template <int H>
__global__ void mlp_prepare_bf16_kernel(float* w) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= H * H) return;
  __bf16* w2 = reinterpret_cast<__bf16*>(reinterpret_cast<char*>(w) + WBf<H>::W2);
  w2[t] = (__bf16)w[WOff<H>::W2 + t];
}

// Row blocks of 16 voxels a wavefront processes at a time.
constexpr int MFMA_MB = 2;

// Transposed products: voxels are the N (column) dimension of both H x H products, so the
// activations of a voxel stay in the lanes of its column c = l % 16 from the inputs to the
// outputs. The C layout gives lane group g = l / 16 the neurons 16 q + 4 g + i (q < H / 16,
// i < 4); the K slots (instruction kb, element j) of a product are mapped onto that same set,
//   slot t = kb J + j  ->  neuron 16 (t / 4) + 4 g + t % 4,
// so the accumulators of one product are the B fragments of the next with no data movement,
// and the layer-1 ReLU masks sit in the lanes of the layer-1 adjoint. Sums over neurons are
// in-lane partial sums plus two cross-group shuffles.
__device__ __forceinline__ int slot_neuron(int t, int g) { return 16 * (t >> 2) + 4 * g + (t & 3); }

template <class P>
__device__ __forceinline__ void put(typename P::frag& f, int j, typename P::elem v) {
  if constexpr (P::J == 1) f = v;
  else f[j] = v;
}

__device__ __forceinline__ float group_sum4(float v) {
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

// A fragments of W2 (rows: output neurons of block r; K: hidden units in slot order), or of
// W2^T (rows: hidden units of block r; K: output neurons in slot order). w2 is row-major
// [out][in] in the element type of P.
template <class P, int H, bool T>
__device__ __forceinline__ void load_w2_frags(const typename P::elem* __restrict__ w2,
                                              typename P::frag (&a)[H / 16][H / P::KS]) {
  const int l = threadIdx.x & 63, c = l & 15, g = l >> 4;
#pragma unroll
  for (int r = 0; r < H / 16; ++r)
#pragma unroll
    for (int kb = 0; kb < H / P::KS; ++kb)
#pragma unroll
      for (int j = 0; j < P::J; ++j) {
        const int u = slot_neuron(kb * P::J + j, g), row = 16 * r + c;
        put<P>(a[r][kb], j, T ? w2[(size_t)u * H + row] : w2[(size_t)row * H + u]);
      }
}

// Raw inputs (d0, d1, d2) of the MB voxel columns of a group; past the end the last voxel is
// read (its results are not stored).
template <int MB>
__device__ __forceinline__ void load_inputs(const float* __restrict__ d0,
                                            const float* __restrict__ d1,
                                            const float* __restrict__ d2, size_t v0, size_t n,
                                            float (&in)[MB][3]) {
  const int c = threadIdx.x & 15;
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) {
    size_t v = v0 + 16 * mb + c;
    v = v < n ? v : n - 1;
    in[mb][0] = d0[v];
    in[mb][1] = d1[v];
    in[mb][2] = d2[v];
  }
}

// Layer 1 as B fragments (K slots = hidden units, N = voxels) and its ReLU mask (bit t).
template <class P, int H>
__device__ __forceinline__ void h1_frags(const float* sw, const float (&in)[3],
                                         typename P::frag (&b)[H / P::KS], uint32_t& mask) {
  const int g = (threadIdx.x & 63) >> 4;
  const float f0 = in[0], f1 = in[1], f2 = in[1] - in[2];
  mask = 0;
#pragma unroll
  for (int kb = 0; kb < H / P::KS; ++kb)
#pragma unroll
    for (int j = 0; j < P::J; ++j) {
      const int t = kb * P::J + j, k = slot_neuron(t, g);
      const float4 r = l1_row<H>(sw, k);
      const float a1 = r.x * f0 + r.y * f1 + r.z * f2 + r.w;
      P::set(b[kb], j, fmaxf(a1, 0.f));
      mask |= (a1 > 0.f ? 1u : 0u) << t;
    }
}

// acc[r] = sum_kb A[r][kb] B[kb] (16 x 16 blocks r of the output neurons, one voxel block).
template <class P, int H>
__device__ __forceinline__ void product(const typename P::frag (&a)[H / 16][H / P::KS],
                                        const typename P::frag (&b)[H / P::KS],
                                        floatx4_t (&acc)[H / 16]) {
#pragma unroll
  for (int r = 0; r < H / 16; ++r) {
    floatx4_t x = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kb = 0; kb < H / P::KS; ++kb) x = P::mma(a[r][kb], b[kb], x);
    acc[r] = x;
  }
}

// y = W3 relu(a2 + b2) + b3 for the voxel of this lane's column (on all four lane groups).
template <int H>
__device__ __forceinline__ float out_layer(const float* sw, const floatx4_t (&acc)[H / 16]) {
  using S = SOff<H>;
  const int g = (threadIdx.x & 63) >> 4;
  float p = 0.f;
#pragma unroll
  for (int q = 0; q < H / 16; ++q)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float2 r = l2_row<H>(sw, 16 * q + 4 * g + i);
      p += r.y * fmaxf(acc[q][i] + r.x, 0.f);
    }
  return group_sum4(p) + sw[S::B3];
}

// W2 in the element type of P, row-major [out][in]: the BF16 copy after the FP32 block, or
// (FP32) the block's own W2.
template <class P, int H>
__device__ __forceinline__ const typename P::elem* w2_rows(const float* w) {
  if constexpr (sizeof(typename P::elem) == 2)
    return reinterpret_cast<const typename P::elem*>(reinterpret_cast<const char*>(w) + WBf<H>::W2);
  else
    return reinterpret_cast<const typename P::elem*>(w + WOff<H>::W2);
}

// Persistent: each wavefront walks groups of 16 MB voxels (wave, wave + all waves, ...) with
// the small FP32 weights in LDS and the W2 fragments in registers, loaded once; the inputs
// of the next group are fetched while the current one is computed.
template <class P, int H>
__global__ __launch_bounds__(TB) void mlp_fwd_mx_kernel(const float* __restrict__ d0,
                                                        const float* __restrict__ d1,
                                                        const float* __restrict__ d2, size_t n,
                                                        const float* __restrict__ w,
                                                        float* __restrict__ mass) {
  using S = SOff<H>;
  constexpr int MB = MFMA_MB, GV = 16 * MB;  // voxels per group
  __shared__ __attribute__((aligned(16))) float sw[S::SIZE];
  load_small_weights<H>(sw, w);
  if (n == 0) return;
  const int l = threadIdx.x & 63;
  typename P::frag aw[H / 16][H / P::KS];
  load_w2_frags<P, H, false>(w2_rows<P, H>(w), aw);
  const size_t groups = (n + GV - 1) / GV;
  const size_t nwaves = (size_t)gridDim.x * (TB / 64);
  size_t gi = (size_t)blockIdx.x * (TB / 64) + (threadIdx.x >> 6);
  float nxt[MB][3];
  load_inputs<MB>(d0, d1, d2, gi * GV, n, nxt);
  for (; gi < groups; gi += nwaves) {
    const size_t v0 = gi * GV;
    float in[MB][3];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
      for (int q = 0; q < 3; ++q) in[mb][q] = nxt[mb][q];
    load_inputs<MB>(d0, d1, d2, v0 + nwaves * GV, n, nxt);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      typename P::frag b[H / P::KS];
      uint32_t mask;
      const float* ws = lds_fence<P, H>(sw);
      h1_frags<P, H>(ws, in[mb], b, mask);
      floatx4_t acc[H / 16];
      product<P, H>(aw, b, acc);
      const float y = out_layer<H>(ws, acc);
      const size_t v = v0 + 16 * mb + (l & 15);
      if (l < 16 && v < n) mass[v] = softplus_f(y);
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
  constexpr int MB = MFMA_MB, GV = 16 * MB;  // voxels per group
  constexpr int KB = H / P::KS;
  __shared__ __attribute__((aligned(16))) float sw[S::SIZE];
  load_small_weights<H>(sw, w);
  if (n == 0) return;
  const int l = threadIdx.x & 63, c = l & 15, g = l >> 4;
  typename P::frag aw[H / 16][KB], at[H / 16][KB];
  load_w2_frags<P, H, false>(w2_rows<P, H>(w), aw);
  load_w2_frags<P, H, true>(w2_rows<P, H>(w), at);
  const size_t groups = (n + GV - 1) / GV;
  const size_t nwaves = (size_t)gridDim.x * (TB / 64);
  size_t gi = (size_t)blockIdx.x * (TB / 64) + (threadIdx.x >> 6);
  float nxt[MB][3], nmb[MB];
  load_inputs<MB>(d0, d1, d2, gi * GV, n, nxt);
#pragma unroll
  for (int mb = 0; mb < MB; ++mb) {
    const size_t v = gi * GV + 16 * mb + c;
    nmb[mb] = mbar[v < n ? v : n - 1];
  }
  for (; gi < groups; gi += nwaves) {
    const size_t v0 = gi * GV;
    float in[MB][3], mbr[MB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
#pragma unroll
      for (int q = 0; q < 3; ++q) in[mb][q] = nxt[mb][q];
      mbr[mb] = nmb[mb];
    }
    load_inputs<MB>(d0, d1, d2, v0 + nwaves * GV, n, nxt);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      const size_t v = v0 + nwaves * GV + 16 * mb + c;
      nmb[mb] = mbar[v < n ? v : n - 1];
    }
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
      const size_t v = v0 + 16 * mb + c;
      typename P::frag b[KB];
      uint32_t mask;
      const float* ws = lds_fence<P, H>(sw);
      h1_frags<P, H>(ws, in[mb], b, mask);
      floatx4_t acc[H / 16];
      product<P, H>(aw, b, acc);
      const float y = out_layer<H>(ws, acc);
      const float yb = v < n ? mbr[mb] * sigmoid_f(y) : 0.f;
      // a2bar = ybar W3 [a2 > 0] as B fragments (K slots = output neurons)
#pragma unroll
      for (int kb = 0; kb < KB; ++kb)
#pragma unroll
        for (int j = 0; j < P::J; ++j) {
          const int t = kb * P::J + j, q = t >> 2, i = t & 3;
          const float2 r = l2_row<H>(ws, 16 * q + 4 * g + i);
          P::set(b[kb], j, acc[q][i] + r.x > 0.f ? yb * r.y : 0.f);
        }
      // h1bar = W2^T a2bar; a1bar = h1bar [a1 > 0]; fbar = W1^T a1bar
      product<P, H>(at, b, acc);
      float p0 = 0.f, p1 = 0.f, p2 = 0.f;
#pragma unroll
      for (int q = 0; q < H / 16; ++q)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int t = 4 * q + i, k = 16 * q + 4 * g + i;
          const float hb = (mask >> t) & 1u ? acc[q][i] : 0.f;
          const float4 r = l1_row<H>(ws, k);
          p0 += r.x * hb;
          p1 += r.y * hb;
          p2 += r.z * hb;
        }
      p0 = group_sum4(p0);
      p1 = group_sum4(p1);
      p2 = group_sum4(p2);
      if (l < 16 && v < n) {
        g0[v] = p0;
        g12[v] = p1 + p2;
        g2[v] = p2;
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
  xd[v] = logf(mtr[v] + (float)prm[b * NPRM + 0]);
}

// Per-cell noise (Eq. probnoise; Sec. 5.1: mu_N and sigma_N depend on the smoothed data
// mass at the cell): linear interpolation of the table (nodes t ascending in
// log(M_R,data), values mu and sigma; constant beyond the end nodes) at log(M_R,data), in
// FP64. Writes mu_N and 1 / (2 sigma_N). tab: [3][NOISE_MAX] doubles (t, mu, sigma).
__global__ void noise_fields_kernel(const float* __restrict__ mrd, size_t total,
                                    const double* __restrict__ tab, int k,
                                    float* __restrict__ nmu, float* __restrict__ nw) {
  const size_t v = (size_t)blockIdx.x * TB + threadIdx.x;
  if (v >= total) return;
  const double* t = tab;
  const double* mu = tab + NOISE_MAX;
  const double* sg = tab + 2 * NOISE_MAX;
  const double m = mrd[v];
  const double x = m > 0.0 ? log(m) : -INFINITY;
  double a, s;
  if (!(x > t[0])) {
    a = mu[0];
    s = sg[0];
  } else if (!(x < t[k - 1])) {
    a = mu[k - 1];
    s = sg[k - 1];
  } else {
    int j = 0;
    while (j + 2 < k && !(x < t[j + 1])) ++j;  // t[j] <= x < t[j + 1]
    const double f = (x - t[j]) / (t[j + 1] - t[j]);
    a = mu[j] + f * (mu[j + 1] - mu[j]);
    s = sg[j] + f * (sg[j + 1] - sg[j]);
  }
  nmu[v] = (float)a;
  nw[v] = (float)(0.5 / s);
}

// r = (mu + log(MR + M0) - x_data) / (2 sigma_N), with per-cell mu_N and 1 / (2 sigma_N)
// when nmu / nw are given.
__global__ void residual_kernel(const float* __restrict__ mr, const float* __restrict__ xd,
                                size_t per_item, int batch, const double* __restrict__ prm,
                                const float* __restrict__ nmu, const float* __restrict__ nw,
                                float* __restrict__ r) {
  const size_t v = (size_t)blockIdx.x * TB + threadIdx.x;
  if (v >= per_item * batch) return;
  const int b = (int)(v / per_item);
  const float M0 = (float)prm[b * NPRM + 0];
  const float mu = nmu ? nmu[v] : (float)prm[b * NPRM + 1];
  const float inv2s = nw ? nw[v] : (float)(0.5 / prm[b * NPRM + 2]);
  r[v] = (mu + logf(mr[v] + M0) - xd[v]) * inv2s;
}

// MRbar = rbar / (2 sigma_N (MR + M0))
__global__ void mrbar_kernel(const float* __restrict__ rbar, const float* __restrict__ mr,
                             size_t per_item, int batch, const double* __restrict__ prm,
                             const float* __restrict__ nw, float* __restrict__ out) {
  const size_t v = (size_t)blockIdx.x * TB + threadIdx.x;
  if (v >= per_item * batch) return;
  const int b = (int)(v / per_item);
  const float M0 = (float)prm[b * NPRM + 0];
  const float inv2s = nw ? nw[v] : (float)(0.5 / prm[b * NPRM + 2]);
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
  // an item whose parameters failed the device-side check reports a NaN loss
  const double bad = prm[b * NPRM + PRM_VALID] != 0.0 ? 0.0 : __builtin_nan("");
  loss_out[3 * b + 0] = prm[b * NPRM + 5] * prior[b] + data[b] + bad;
  loss_out[3 * b + 1] = prior[b] + bad;
  loss_out[3 * b + 2] = data[b] + bad;
}

// ---------------------------------------------------------------- loss parameters
// Host parameters arrive as kernel arguments (copied at launch), so the host array need not
// outlive the call and nothing waits for the copy.
__global__ void params_store_kernel(ParamChunk c, double* __restrict__ prm) {
  const int i = threadIdx.x;
  if (i < c.count * NPRM) prm[(size_t)c.b0 * NPRM + i] = c.v[i];
}

// Parameters from device memory (PMR_LOSS_FIELDS doubles per item, the field order of the
// public struct), checked here: an item that fails the check is stored with its validity
// slot 0, which makes its loss NaN.
__global__ void params_from_device_kernel(const double* __restrict__ src, int batch,
                                          int density_l2, int halo_two,
                                          double* __restrict__ prm) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  double v[PMR_LOSS_FIELDS];
#pragma unroll
  for (int i = 0; i < PMR_LOSS_FIELDS; ++i) v[i] = src[(size_t)b * PMR_LOSS_FIELDS + i];
  bool ok = v[2] > 0.0 && v[2] < INFINITY && (density_l2 || (v[0] > 0.0 && v[0] < INFINITY)) &&
            v[3] >= 0.0 && v[3] < INFINITY && v[4] >= 0.0 && v[4] < INFINITY &&
            isfinite(v[1]) && isfinite(v[5]);
  if (halo_two) ok = ok && v[6] > 0.0 && v[6] < INFINITY;
#pragma unroll
  for (int i = 0; i < PMR_LOSS_FIELDS; ++i) prm[(size_t)b * NPRM + i] = v[i];
  prm[(size_t)b * NPRM + PRM_VALID] = ok ? 1.0 : 0.0;
}

__global__ void noise_table_store_kernel(NoiseTable t, double* __restrict__ tab) {
  for (int i = threadIdx.x; i < 3 * NOISE_MAX; i += blockDim.x) tab[i] = t.v[i];
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
  // FP32 block, then the BF16 W2 (16-byte aligned)
  return ((size_t)6 * H + (size_t)H * H + 1 + 3) / 4 * 4 + ((size_t)H * H + 1) / 2 + 4;
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
                     const double* prm, const float* nmu, const float* nw, float* r,
                     hipStream_t s) {
  residual_kernel<<<grid1(per_item * batch), TB, 0, s>>>(mr, xd, per_item, batch, prm, nmu, nw,
                                                         r);
}
void launch_mrbar(const float* rbar, const float* mr, size_t per_item, int batch,
                  const double* prm, const float* nw, float* out, hipStream_t s) {
  mrbar_kernel<<<grid1(per_item * batch), TB, 0, s>>>(rbar, mr, per_item, batch, prm, nw, out);
}
void launch_noise_fields(const float* mrd, size_t total, const double* tab, int k, float* nmu,
                         float* nw, hipStream_t s) {
  noise_fields_kernel<<<grid1(total), TB, 0, s>>>(mrd, total, tab, k, nmu, nw);
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

void launch_params_store(const double* host, int batch, double* prm, hipStream_t s) {
  for (int b0 = 0; b0 < batch; b0 += PRM_CHUNK) {
    ParamChunk c;
    c.b0 = b0;
    c.count = batch - b0 < PRM_CHUNK ? batch - b0 : PRM_CHUNK;
    for (int i = 0; i < c.count * NPRM; ++i) c.v[i] = host[(size_t)b0 * NPRM + i];
    params_store_kernel<<<1, PRM_CHUNK * NPRM, 0, s>>>(c, prm);
  }
}

void launch_params_from_device(const double* src, int batch, int density_l2, int halo_two,
                               double* prm, hipStream_t s) {
  params_from_device_kernel<<<(batch + 63) / 64, 64, 0, s>>>(src, batch, density_l2, halo_two,
                                                             prm);
}

void launch_noise_table_store(const double* host, double* tab, hipStream_t s) {
  NoiseTable t;
  for (int i = 0; i < 3 * NOISE_MAX; ++i) t.v[i] = host[i];
  noise_table_store_kernel<<<1, 256, 0, s>>>(t, tab);
}

}  // namespace pmr
