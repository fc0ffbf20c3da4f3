// Second-order Lagrangian initial conditions (Sec. 3: the simulations start from 2LPT):
// the pointwise parts. With phi_ab the second derivatives of the potential of the linear
// field (computed by the Hessian x-pass operator), the second-order source is
//   S = phi_xx phi_yy + phi_xx phi_zz + phi_yy phi_zz - phi_xy^2 - phi_xz^2 - phi_yz^2,
// and the adjoint of that map sends S_bar to
//   phi_bar_xx = (phi_yy + phi_zz) S_bar, phi_bar_yy = (phi_xx + phi_zz) S_bar,
//   phi_bar_zz = (phi_xx + phi_yy) S_bar, phi_bar_ab = -2 phi_ab S_bar (a != b).
// Fields are [B][6][np^3] in the pair order xx, yy, zz, xy, xz, yz; S and S_bar are one
// field per item at a caller-given item stride. Both kernels stream HBM (28 and 52 bytes per
// lattice site) with 16-byte accesses; np^3 is a multiple of 4.
#include "../../include/pmr.h"
#include "pmr_internal.h"

namespace pmr {
namespace {

constexpr int TB = 256;

__device__ __forceinline__ float4 ld4(const float* p) { return *reinterpret_cast<const float4*>(p); }
__device__ __forceinline__ void st4(float* p, float4 v) { *reinterpret_cast<float4*>(p) = v; }

// S from the six phi (the products summed in FP64: the terms cancel in voids).
__global__ __launch_bounds__(TB) void lpt2_source_kernel(const float* __restrict__ phi,
                                                         int log_np3, size_t quads,
                                                         float* __restrict__ S,
                                                         size_t s_item_stride) {
  const size_t g = (size_t)blockIdx.x * TB + threadIdx.x;
  if (g >= quads) return;
  const size_t np3 = (size_t)1 << log_np3;
  const size_t e = g * 4;  // first site of this quad, batch-flattened
  const size_t item = e >> log_np3, id = e & (np3 - 1);
  const float* b = phi + item * 6 * np3 + id;
  const float4 xx = ld4(b), yy = ld4(b + np3), zz = ld4(b + 2 * np3);
  const float4 xy = ld4(b + 3 * np3), xz = ld4(b + 4 * np3), yz = ld4(b + 5 * np3);
  auto src = [](float a, float bb, float c, float d, float f, float h) {
    const double A = a, Bv = bb, C = c, Dv = d, F = f, Hv = h;
    return (float)(A * Bv + A * C + Bv * C - Dv * Dv - F * F - Hv * Hv);
  };
  float4 o;
  o.x = src(xx.x, yy.x, zz.x, xy.x, xz.x, yz.x);
  o.y = src(xx.y, yy.y, zz.y, xy.y, xz.y, yz.y);
  o.z = src(xx.z, yy.z, zz.z, xy.z, xz.z, yz.z);
  o.w = src(xx.w, yy.w, zz.w, xy.w, xz.w, yz.w);
  st4(S + item * s_item_stride + id, o);
}

__global__ __launch_bounds__(TB) void lpt2_phi_bar_kernel(const float* __restrict__ phi,
                                                          const float* __restrict__ Sbar,
                                                          size_t s_item_stride, int log_np3,
                                                          size_t quads,
                                                          float* __restrict__ phibar) {
  const size_t g = (size_t)blockIdx.x * TB + threadIdx.x;
  if (g >= quads) return;
  const size_t np3 = (size_t)1 << log_np3;
  const size_t e = g * 4;
  const size_t item = e >> log_np3, id = e & (np3 - 1);
  const size_t off = item * 6 * np3 + id;
  const float* b = phi + off;
  float* o = phibar + off;
  const float4 s = ld4(Sbar + item * s_item_stride + id);
  const float4 xx = ld4(b), yy = ld4(b + np3), zz = ld4(b + 2 * np3);
  st4(o, make_float4((yy.x + zz.x) * s.x, (yy.y + zz.y) * s.y, (yy.z + zz.z) * s.z,
                     (yy.w + zz.w) * s.w));
  st4(o + np3, make_float4((xx.x + zz.x) * s.x, (xx.y + zz.y) * s.y, (xx.z + zz.z) * s.z,
                           (xx.w + zz.w) * s.w));
  st4(o + 2 * np3, make_float4((xx.x + yy.x) * s.x, (xx.y + yy.y) * s.y, (xx.z + yy.z) * s.z,
                               (xx.w + yy.w) * s.w));
#pragma unroll
  for (int q = 3; q < 6; ++q) {
    const float4 v = ld4(b + q * np3);
    st4(o + q * np3, make_float4(-2.f * v.x * s.x, -2.f * v.y * s.y, -2.f * v.z * s.z,
                                 -2.f * v.w * s.w));
  }
}

}  // namespace

void launch_lpt2_source(const float* phi, int batch, int log_np3, float* S, size_t s_item_stride,
                        hipStream_t s) {
  const size_t quads = ((size_t)batch << log_np3) / 4;
  lpt2_source_kernel<<<(unsigned)((quads + TB - 1) / TB), TB, 0, s>>>(phi, log_np3, quads, S,
                                                                      s_item_stride);
}

void launch_lpt2_phi_bar(const float* phi, const float* Sbar, size_t s_item_stride, int batch,
                         int log_np3, float* phibar, hipStream_t s) {
  const size_t quads = ((size_t)batch << log_np3) / 4;
  lpt2_phi_bar_kernel<<<(unsigned)((quads + TB - 1) / TB), TB, 0, s>>>(phi, Sbar, s_item_stride,
                                                                       log_np3, quads, phibar);
}

}  // namespace pmr
