// 3-D real FFTs of n^3 meshes (n = 16..512, power of two), staged in LDS.
//
// Layout: real fields [n][n][n] row-major (z fastest); spectra [n][n][n/2+1] interleaved
// complex (numpy rfftn layout). Forward transform unnormalised; every inverse path
// carries its 1/n^3 inside the k-space operator of the outermost-axis pass.
//
// The transform is three passes, each reading and writing the whole array once:
//   z pass : contiguous rows; r2c as an n/2-point complex FFT of (x_even + i x_odd)
//            followed by the standard split step (c2r: the inverse split, then the FFT).
//   y pass : lines of stride n/2+1; a workgroup owns 16 consecutive kz columns of one
//            x-plane, so every global access is a 128-byte run.
//   x pass : lines of stride n(n/2+1); same tiling. This pass sees complete k-vectors,
//            so the k-space operators (force, Gaussian smoothing, their adjoints, the
//            Zel'dovich displacement and the gradient assembly) run inside it,
//            between a forward and an inverse transform, without extra HBM traffic.
// Each line transform is a self-sorting Stockham FFT (radix 8, then 4 or 2) in LDS;
// twiddles are evaluated once per workgroup in FP64 and rounded to FP32.
#pragma once
#include "pmr_internal.h"
#include "twiddle.h"

namespace pmr {


namespace {

#include "paint_kernels.h"

constexpr int NT = 256;   // threads per FFT workgroup (4 waves)
constexpr int PCOL = 16;  // columns per strided-pass tile (16 complex = 128 B)

// ---------------------------------------------------------------- butterflies
template <int DIR>
__device__ __forceinline__ void bfly2(float2* u) {
  float2 a = u[0];
  u[0] = cadd(a, u[1]);
  u[1] = csub(a, u[1]);
}

template <int DIR>
__device__ __forceinline__ void bfly4(float2& a0, float2& a1, float2& a2, float2& a3) {
  float2 t0 = cadd(a0, a2), t1 = csub(a0, a2);
  float2 t2 = cadd(a1, a3), t3 = cmul_i<DIR>(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

template <int DIR>
__device__ __forceinline__ void bfly8(float2* u) {
  const float c = 0.70710678118654752440f;
  bfly4<DIR>(u[0], u[2], u[4], u[6]);
  bfly4<DIR>(u[1], u[3], u[5], u[7]);
  // odd half times omega_8^q, omega_8 = exp(DIR * 2 pi i / 8)
  float2 o1 = u[3], o2 = u[5], o3 = u[7];
  o1 = make_float2(c * (o1.x - DIR * o1.y), c * (o1.y + DIR * o1.x));
  o2 = cmul_i<DIR>(o2);
  o3 = make_float2(c * (-o3.x - DIR * o3.y), c * (DIR * o3.x - o3.y));
  float2 e0 = u[0], e1 = u[2], e2 = u[4], e3 = u[6], o0 = u[1];
  u[0] = cadd(e0, o0);
  u[4] = csub(e0, o0);
  u[1] = cadd(e1, o1);
  u[5] = csub(e1, o1);
  u[2] = cadd(e2, o2);
  u[6] = csub(e2, o2);
  u[3] = cadd(e3, o3);
  u[7] = csub(e3, o3);
}

template <int R, int DIR>
__device__ __forceinline__ void bfly(float2* u) {
  if constexpr (R == 2) bfly2<DIR>(u);
  if constexpr (R == 4) bfly4<DIR>(u[0], u[1], u[2], u[3]);
  if constexpr (R == 8) bfly8<DIR>(u);
}

// ---------------------------------------------------------------- Stockham stage
// M-point transforms of LINES lines held in LDS; point n of line l at lds[n*SN + l*SL], or at
// lds[n + (n >> 5) + l*SL] when PAD (SN = 1): one padding slot every 32 points keeps the
// strided butterfly writes of the first stages on distinct LDS banks.
// Stage with radix R after earlier stages of total radix PREV: butterfly i (0..M/R-1)
// reads points i + r M/R, twiddles by w^(r k M / (PREV R)) with k = i mod PREV, and
// writes point (i - k) R + k + r PREV. Twiddle table: tw[j * TWS] = exp(-2 pi i j / M).
template <int SN, bool PAD>
__device__ __forceinline__ int lpos(int n) {
  if constexpr (PAD) return n + (n >> 5);
  return n * SN;
}

template <int M, int R, int PREV, int LINES, int SN, int SL, int TWS, int DIR, int NTH, bool PAD>
__device__ __forceinline__ void stockham_stage(float2* lds, const float2* tw) {
  static_assert(!PAD || SN == 1, "padding applies to unit-stride lines");
  constexpr int NB = (M / R) * LINES;
  constexpr int PER = (NB + NTH - 1) / NTH;
  float2 u[PER][R];
  int ii[PER], ll[PER];
  const int t = threadIdx.x;
#pragma unroll
  for (int m = 0; m < PER; ++m) {
    const int b = t + m * NTH;
    ii[m] = -1;
    if (NB % NTH == 0 || b < NB) {
      int i, l;
      if constexpr (SL == 1) {
        l = b % LINES;
        i = b / LINES;
      } else {
        i = b % (M / R);
        l = b / (M / R);
      }
      ii[m] = i;
      ll[m] = l;
#pragma unroll
      for (int r = 0; r < R; ++r) u[m][r] = lds[lpos<SN, PAD>(i + r * (M / R)) + l * SL];
    }
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < PER; ++m) {
    if (NB % NTH == 0 || ii[m] >= 0) {
      const int i = ii[m], l = ll[m];
      const int k = i & (PREV - 1);
      if constexpr (PREV > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          float2 w = tw[r * k * (M / (PREV * R)) * TWS];
          if (DIR > 0) w.y = -w.y;
          u[m][r] = cmul(u[m][r], w);
        }
      }
      bfly<R, DIR>(u[m]);
      const int j0 = (i - k) * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) lds[lpos<SN, PAD>(j0 + r * PREV) + l * SL] = u[m][r];
    }
  }
  __syncthreads();
}

// Full M-point transform. RMAX = 8: radix-8 stages, then one radix-4 or radix-2 stage;
// RMAX = 4: radix-4 stages, then one radix-2 stage (more LDS round trips with fewer live
// values per thread; the autotuner chooses per pass).
template <int M, int LINES, int SN, int SL, int TWS, int DIR, int NTH = NT, bool PAD = false,
          int RMAX = 8>
__device__ __forceinline__ void fft_lds(float2* lds, const float2* tw) {
  static_assert(M >= 2 && (M & (M - 1)) == 0, "power of two");
  static_assert(RMAX == 8 || RMAX == 4, "radix-8 or radix-4 plan");
  static_assert(M <= 512, "at most 512 points per line");
  if constexpr (RMAX == 8) {
    if constexpr (M >= 8) stockham_stage<M, 8, 1, LINES, SN, SL, TWS, DIR, NTH, PAD>(lds, tw);
    if constexpr (M >= 64) stockham_stage<M, 8, 8, LINES, SN, SL, TWS, DIR, NTH, PAD>(lds, tw);
    if constexpr (M >= 512) stockham_stage<M, 8, 64, LINES, SN, SL, TWS, DIR, NTH, PAD>(lds, tw);
    constexpr int P8 = M >= 512 ? 512 : M >= 64 ? 64 : M >= 8 ? 8 : 1;
    constexpr int REM = M / P8;
    if constexpr (REM == 4) stockham_stage<M, 4, P8, LINES, SN, SL, TWS, DIR, NTH, PAD>(lds, tw);
    if constexpr (REM == 2) stockham_stage<M, 2, P8, LINES, SN, SL, TWS, DIR, NTH, PAD>(lds, tw);
  } else {
    if constexpr (M >= 4) stockham_stage<M, 4, 1, LINES, SN, SL, TWS, DIR, NTH, PAD>(lds, tw);
    if constexpr (M >= 16) stockham_stage<M, 4, 4, LINES, SN, SL, TWS, DIR, NTH, PAD>(lds, tw);
    if constexpr (M >= 64) stockham_stage<M, 4, 16, LINES, SN, SL, TWS, DIR, NTH, PAD>(lds, tw);
    if constexpr (M >= 256) stockham_stage<M, 4, 64, LINES, SN, SL, TWS, DIR, NTH, PAD>(lds, tw);
    constexpr int P4 = M >= 256 ? 256 : M >= 64 ? 64 : M >= 16 ? 16 : M >= 4 ? 4 : 1;
    if constexpr (M / P4 == 2) stockham_stage<M, 2, P4, LINES, SN, SL, TWS, DIR, NTH, PAD>(lds, tw);
  }
}

// exp(-2 pi i j / N) for j < N: copied from the compile-time table (twiddle.h).
template <int N>
__device__ constexpr TwTable<N> kTw = make_tw_table<N>();

template <int N, int NTH = NT>
__device__ __forceinline__ void make_twiddles(float2* tw) {
  for (int j = threadIdx.x; j < N; j += NTH) {
    const TwEntry e = kTw<N>.v[j];
    tw[j] = make_float2(e.re, e.im);
  }
}

// ---------------------------------------------------------------- k-space factors
// k_a = kf m of storage index i along one axis (m = i for i <= N / 2, else i - N; the half
// kz axis needs no wrap), zero on the Nyquist plane as in the force operator's gradient factors.
template <int N>
__device__ __forceinline__ float axis_coef(int i, float kf) {
  const int m = wavenumber(i, N);
  return (m == N / 2 || m == -N / 2) ? 0.f : kf * m;
}

// ---------------------------------------------------------------- z pass, r2c
template <int N>
struct ZTile {
  static constexpr int H = N / 2;                        // complex points per row
  static constexpr int ROWS = (2048 / H) > 0 ? 2048 / H : 1;
  static constexpr int PITCH = H + H / 32 + 1;           // LDS row pitch (complex, padded)
};

// LDS slot of point k of a z-pass row (one padding slot every 32 points, see lpos).
__device__ __forceinline__ int zk(int k) { return k + (k >> 5); }

// The z passes are tile loops: a workgroup walks tiles blockIdx-remapped, blockIdx + grid, ...
// (tile = one field's group of consecutive rows), prefetching the next tile's input into
// registers while the current one is transformed, and computes its twiddles once.

// Inverse split of one row pair: Z[k] = E + i O with E = X[k] + conj X[H-k] and
// O = (X[k] - conj X[H-k]) conj(W^k), W = e^{-2 pi i / N}; k = 0 combines X[0] and X[H].
template <int H>
__device__ __forceinline__ void inv_split(float2* z, int k, float2 xk, float2 xm, const float2* tw) {
  if (k == 0) {
    z[0] = make_float2(xk.x + xm.x, xk.x - xm.x);  // xk = X[0], xm = X[H] (real parts)
    return;
  }
  {
    float2 E = make_float2(xk.x + xm.x, xk.y - xm.y);
    float2 D = make_float2(xk.x - xm.x, xk.y + xm.y);
    float2 O = cmul(D, cconj(tw[k]));
    z[zk(k)] = make_float2(E.x - O.y, E.y + O.x);
  }
  if (k != H - k) {
    float2 E = make_float2(xm.x + xk.x, xm.y - xk.y);
    float2 D = make_float2(xm.x - xk.x, xm.y + xk.y);
    float2 O = cmul(D, cconj(tw[H - k]));
    z[zk(H - k)] = make_float2(E.x - O.y, E.y + O.x);
  }
}

// in: fields of n^3 reals; out = fields of n*n*(n/2+1) complex (row pitch om.pitch). One tile
// (ROWS rows of one field) per workgroup: measured faster here than a prefetching tile loop.
// Value loaded: a1 * in (+ a2 * in2 if in2) (* scale_dev[field / fields_per_item]).
template <int N>
__global__ __launch_bounds__(NT) void zpass_r2c_kernel(const float* __restrict__ in, FieldMap im,
                                                       const float* __restrict__ in2, float a1,
                                                       float a2, const double* __restrict__ scale_dev,
                                                       float2* __restrict__ out, FieldMap om) {
  using T = ZTile<N>;
  constexpr int H = T::H, ROWS = T::ROWS, PITCH = T::PITCH;
  __shared__ float2 lds[ROWS * PITCH];
  __shared__ float2 tw[N];
  make_twiddles<N>(tw);
  const int field = blockIdx.y;
  const size_t row0 = (size_t)xcd_block(blockIdx.x, gridDim.x) * ROWS;
  const float2* src = reinterpret_cast<const float2*>(in + im.off(field)) + row0 * H;
  const float2* src2 =
      in2 ? reinterpret_cast<const float2*>(in2 + im.off(field)) + row0 * H : nullptr;
  float sc = 1.0f;
  if (scale_dev) sc = (float)scale_dev[field / im.fpi];
  const float b1 = a1 * sc, b2 = a2 * sc;
  for (int e = threadIdx.x; e < ROWS * H; e += NT) {
    float2 v = src[e];
    v.x *= b1;
    v.y *= b1;
    if (src2) {
      float2 w = src2[e];
      v.x += b2 * w.x;
      v.y += b2 * w.y;
    }
    lds[(e / H) * PITCH + zk(e % H)] = v;
  }
  __syncthreads();
  fft_lds<H, ROWS, 1, PITCH, 2, -1, NT, true>(lds, tw);
  // split: X[k] = (Z[k] + conj Z[H-k]) / 2 - i W^k (Z[k] - conj Z[H-k]) / 2, W = e^{-2 pi i/N}
  float2* dst = out + om.off(field) + row0 * om.pitch;
  constexpr int Q = H / 2 + 1;  // pairs (k, H-k) for k = 0..H/2
  for (int e = threadIdx.x; e < ROWS * Q; e += NT) {
    const int r = e / Q, k = e % Q;
    const float2* z = lds + r * PITCH;
    float2* d = dst + (size_t)r * om.pitch;
    if (k == 0) {
      float2 z0 = z[0];
      d[0] = make_float2(z0.x + z0.y, 0.f);
      d[H] = make_float2(z0.x - z0.y, 0.f);
    } else {
      const float2 zv = z[zk(k)], zm = z[zk(H - k)];
      {
        float2 s = make_float2(0.5f * (zv.x + zm.x), 0.5f * (zv.y - zm.y));
        float2 df = make_float2(0.5f * (zv.x - zm.x), 0.5f * (zv.y + zm.y));
        float2 w = tw[k];
        float2 t = cmul(w, df);  // W^k * diff
        d[k] = make_float2(s.x + t.y, s.y - t.x);  // s - i t
      }
      if (k != H - k) {
        float2 s = make_float2(0.5f * (zm.x + zv.x), 0.5f * (zm.y - zv.y));
        float2 df = make_float2(0.5f * (zm.x - zv.x), 0.5f * (zm.y + zv.y));
        float2 w = tw[H - k];
        float2 t = cmul(w, df);
        d[H - k] = make_float2(s.x + t.y, s.y - t.x);
      }
    }
  }
}

// CIC paint fused with the z pass of the following r2c (Sec. 3: the density that feeds the
// force, or the three adjoint channels in the step adjoint): a workgroup owns W * TY
// consecutive target rows of one (item, ix) plane (TY per wavefront, deposited as in the
// paint kernels, into LDS rows already in the z pass's padded complex layout), then
// transforms those rows in place and writes their half spectra. The real mesh never goes
// through HBM. rho - bias only changes X[0] of each row, by bias * N.
template <int N>
constexpr int paint_r2c_ty(int C) {
  int ty = PMR_PAINT_LDS_FLOATS / (N * C);
  if (ty > PMR_PAINT_TY_MAX) ty = PMR_PAINT_TY_MAX;
  if (ty > N / 2) ty = N / 2;
  if (ty > N / (NT / 64)) ty = N / (NT / 64);  // whole workgroups of rows per plane
  int p = 1;
  while (p * 2 <= ty) p *= 2;
  return p;
}

// Store of one spectrum value; STREAM: past the caches (non-temporal), for spectra larger
// than the memory-side cache, whose lines would be evicted before the next pass reads them
// anyway (at 512^3 the fused paints measured 2-5% faster; at 128^3, where the next pass
// finds the spectrum in that cache, slower).
template <bool STREAM>
__device__ __forceinline__ void store_spec(float2* p, float2 v) {
  if constexpr (STREAM) {
    __builtin_nontemporal_store(v.x, &p->x);
    __builtin_nontemporal_store(v.y, &p->y);
  } else {
    *p = v;
  }
}

template <int C, int TY, int N>
__global__ __launch_bounds__(NT) void paint_r2c_kernel(PaintArgs a, float2* __restrict__ out,
                                                       FieldMap om) {
  using T = ZTile<N>;
  constexpr int H = T::H, PITCH = T::PITCH, RP = 2 * PITCH;  // row pitch: complex, floats
  constexpr int W = NT / 64;
  constexpr int LINES = W * TY * C;
  constexpr int BPX = N / (W * TY);  // workgroups per (item, ix) plane
  __shared__ __attribute__((aligned(16))) float acc_all[LINES * RP];
  __shared__ float2 tw[N];
  make_twiddles<N>(tw);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int item = blk / (N * BPX);
  const int rr = blk - item * N * BPX;
  const int ix = rr / BPX;
  const int iyb = (rr - ix * BPX) * (W * TY);  // first row of the workgroup
  float* acc = acc_all + (size_t)w * TY * C * RP;
  for (int i = lane; i < TY * C * RP; i += 64) acc[i] = 0.f;
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_s_waitcnt(0xc07f);
  paint_rows<C, TY, true>(a, item, ix, iyb + w * TY, acc, RP);
  __syncthreads();  // every row of the workgroup deposited; twiddles in place
  float2* lds = reinterpret_cast<float2*>(acc_all);
  fft_lds<H, LINES, 1, PITCH, 2, -1, NT, true>(lds, tw);
  constexpr int Q = H / 2 + 1;  // pairs (k, H-k) for k = 0..H/2
  const float bN = a.bias * (float)N;
  for (int e = threadIdx.x; e < LINES * Q; e += NT) {
    const int line = e / Q, k = e % Q;  // line = (wave * TY + t) * C + c
    const int c = line % C, t = line / C;  // t: row within the workgroup
    const float2* z = lds + line * PITCH;
    float2* d = out + om.off(item * C + c) + ((size_t)ix * N + iyb + t) * om.pitch;
    if (k == 0) {
      const float2 z0 = z[0];
      store_spec<(N >= 512)>(&d[0], make_float2(z0.x + z0.y - bN, 0.f));
      store_spec<(N >= 512)>(&d[H], make_float2(z0.x - z0.y, 0.f));
    } else {
      const float2 zv = z[zk(k)], zm = z[zk(H - k)];
      {
        float2 sm = make_float2(0.5f * (zv.x + zm.x), 0.5f * (zv.y - zm.y));
        float2 df = make_float2(0.5f * (zv.x - zm.x), 0.5f * (zv.y + zm.y));
        float2 t2 = cmul(tw[k], df);
        store_spec<(N >= 512)>(&d[k], make_float2(sm.x + t2.y, sm.y - t2.x));
      }
      if (k != H - k) {
        float2 sm = make_float2(0.5f * (zm.x + zv.x), 0.5f * (zm.y - zv.y));
        float2 df = make_float2(0.5f * (zm.x - zv.x), 0.5f * (zm.y + zv.y));
        float2 t2 = cmul(tw[H - k], df);
        store_spec<(N >= 512)>(&d[H - k], make_float2(sm.x + t2.y, sm.y - t2.x));
      }
    }
  }
}

// Rows per wave TY the fused paint can take at size N with C channels: TY <= N / 2, whole
// workgroups of rows per plane, and the workgroup's padded rows plus twiddles within 160 KB.
template <int N, int C, int TY>
constexpr bool paint_r2c_ty_ok() {
  constexpr int W = NT / 64;
  using T = ZTile<N>;
  return TY <= N / 2 && TY <= N / W &&
         (size_t)W * TY * C * 2 * T::PITCH * 4 + (size_t)N * 8 <= 160 * 1024;
}

template <int C, int TY, int N>
void paint_r2c_launch(const PaintArgs& a, int batch, float2* out, FieldMap om, hipStream_t s) {
  constexpr int W = NT / 64;
  const int blocks = batch * N * (N / (W * TY));
  paint_r2c_kernel<C, TY, N><<<blocks, NT, 0, s>>>(a, out, om);
}

// TY from the tuned table (0: the default rule paint_r2c_ty), falling back to the default
// when the tuned value is not a valid shape.
template <int C, int N>
void paint_r2c(const PaintArgs& a, int batch, float2* out, FieldMap om, hipStream_t s) {
  const int want = get_paint_rows(N, C);
#define TYCASE(T)                                                  \
  if constexpr (paint_r2c_ty_ok<N, C, T>())                        \
    if (want == T) {                                               \
      paint_r2c_launch<C, T, N>(a, batch, out, om, s);             \
      return;                                                      \
    }
  TYCASE(1) TYCASE(2) TYCASE(4) TYCASE(8) TYCASE(16)
#undef TYCASE
  paint_r2c_launch<C, paint_r2c_ty<N>(C), N>(a, batch, out, om, s);
}

// Row pairs (k, H - k) of a c2r tile held in registers: pair e = threadIdx + m NT of the
// tile's LINES * Q pairs (line = e / Q, k = e % Q).
template <int H, int LINES>
struct PairRegs {
  static constexpr int Q = H / 2 + 1;
  static constexpr int PER = (LINES * Q + NT - 1) / NT;
  float2 a[PER], b[PER];
};

// in: fields of n*n*(n/2+1) complex (row pitch im.pitch); out: fields of n^3 reals = the
// unnormalised inverse transform along z of each row (imaginary parts of the kz = 0 and n/2
// entries ignored). Optional epilogue: out += add.
template <int N>
__global__ __launch_bounds__(NT) void zpass_c2r_kernel(const float2* __restrict__ in, FieldMap im,
                                                       float* __restrict__ out, FieldMap om,
                                                       const float* __restrict__ add,
                                                       int tiles_per_field, int ntiles) {
  using T = ZTile<N>;
  constexpr int H = T::H, ROWS = T::ROWS, PITCH = T::PITCH;
  using PR = PairRegs<H, ROWS>;
  constexpr int Q = PR::Q;
  __shared__ float2 lds[ROWS * PITCH];
  __shared__ float2 tw[N];
  make_twiddles<N>(tw);
  auto load = [&](int t, PR& r) {
    const int field = t / tiles_per_field;
    const size_t row0 = (size_t)(t % tiles_per_field) * ROWS;
    const float2* src = in + im.off(field) + row0 * im.pitch;
#pragma unroll
    for (int m = 0; m < PR::PER; ++m) {
      const int e = threadIdx.x + m * NT;
      if (e < ROWS * Q) {
        const int rr = e / Q, k = e % Q;
        const float2* x = src + (size_t)rr * im.pitch;
        r.a[m] = x[k];
        r.b[m] = x[H - k];
      }
    }
  };
  int tau = xcd_block(blockIdx.x, gridDim.x);
  PR pre;
  load(tau, pre);
  __syncthreads();  // twiddles
  for (;;) {
#pragma unroll
    for (int m = 0; m < PR::PER; ++m) {
      const int e = threadIdx.x + m * NT;
      if (e < ROWS * Q) inv_split<H>(lds + (e / Q) * PITCH, e % Q, pre.a[m], pre.b[m], tw);
    }
    __syncthreads();
    const int next = tau + gridDim.x;
    if (next < ntiles) load(next, pre);
    fft_lds<H, ROWS, 1, PITCH, 2, +1, NT, true>(lds, tw);
    const int field = tau / tiles_per_field;
    const size_t row0 = (size_t)(tau % tiles_per_field) * ROWS;
    float2* dst = reinterpret_cast<float2*>(out + om.off(field)) + row0 * H;
    const float2* ad = add ? reinterpret_cast<const float2*>(add + om.off(field)) + row0 * H : nullptr;
    static_assert((ROWS * H) % NT == 0, "whole rows per thread sweep");
#pragma unroll
    for (int m = 0; m < ROWS * H / NT; ++m) {
      const int e = threadIdx.x + m * NT;
      float2 v = lds[(e / H) * PITCH + zk(e % H)];
      if (ad) {
        const float2 w = ad[e];
        v.x += w.x;
        v.y += w.y;
      }
      store_spec<(N >= 512)>(&dst[e], v);
    }
    if (next >= ntiles) break;
    __syncthreads();
    tau = next;
  }
}

// Three fields per item (the components of a vector field) -> one interleaved mesh of
// (f0, f1, f2) cells [item][n^3]: a CIC readout of all three components at a corner is then
// one 12-byte load instead of three loads from three meshes. Same transform as
// zpass_c2r_kernel.
template <int N>
struct ZTile3 {
  static constexpr int R = ZTile<N>::ROWS / 2 > 0 ? ZTile<N>::ROWS / 2 : 1;  // rows per field
};

template <int N>
__global__ __launch_bounds__(NT) void zpass_c2r3_kernel(const float2* __restrict__ in, FieldMap im,
                                                        Vec3* __restrict__ out,
                                                        size_t out_item_stride,
                                                        int tiles_per_item, int ntiles) {
  using T = ZTile<N>;
  constexpr int H = T::H, PITCH = T::PITCH, R = ZTile3<N>::R;
  using PR = PairRegs<H, 3 * R>;
  constexpr int Q = PR::Q;
  __shared__ float2 lds[3 * R * PITCH];
  __shared__ float2 tw[N];
  make_twiddles<N>(tw);
  auto load = [&](int t, PR& r) {
    const int item = t / tiles_per_item;
    const size_t row0 = (size_t)(t % tiles_per_item) * R;
#pragma unroll
    for (int m = 0; m < PR::PER; ++m) {
      const int e = threadIdx.x + m * NT;
      if (e < 3 * R * Q) {
        const int line = e / Q, k = e % Q;  // line = component * R + row
        const int f = line / R, rr = line % R;
        const float2* x = in + im.off(item * 3 + f) + (row0 + rr) * im.pitch;
        r.a[m] = x[k];
        r.b[m] = x[H - k];
      }
    }
  };
  int tau = xcd_block(blockIdx.x, gridDim.x);
  PR pre;
  load(tau, pre);
  __syncthreads();  // twiddles
  for (;;) {
#pragma unroll
    for (int m = 0; m < PR::PER; ++m) {
      const int e = threadIdx.x + m * NT;
      if (e < 3 * R * Q) inv_split<H>(lds + (e / Q) * PITCH, e % Q, pre.a[m], pre.b[m], tw);
    }
    __syncthreads();
    const int next = tau + gridDim.x;
    if (next < ntiles) load(next, pre);
    fft_lds<H, 3 * R, 1, PITCH, 2, +1, NT, true>(lds, tw);
    const int item = tau / tiles_per_item;
    const size_t row0 = (size_t)(tau % tiles_per_item) * R;
    Vec3* dst = out + item * out_item_stride + row0 * N;
    const float* l = reinterpret_cast<const float*>(lds);
    static_assert((R * N) % NT == 0, "whole rows per thread sweep");
#pragma unroll
    for (int m = 0; m < R * N / NT; ++m) {
      const int e = threadIdx.x + m * NT;
      const int r = e / N, zz = e % N;
      const int q = 2 * zk(zz >> 1) + (zz & 1);  // float slot of real point zz
      // non-temporal: the force mesh is read only by the kick that follows the whole pass
      __builtin_nontemporal_store(l[(0 * R + r) * 2 * PITCH + q], &dst[e].x);
      __builtin_nontemporal_store(l[(1 * R + r) * 2 * PITCH + q], &dst[e].y);
      __builtin_nontemporal_store(l[(2 * R + r) * 2 * PITCH + q], &dst[e].z);
    }
    if (next >= ntiles) break;
    __syncthreads();
    tau = next;
  }
}

// ---------------------------------------------------------------- strided passes
// Tile: PC consecutive kz columns (from kz0) of the N points of one line family.
// Element (n, l) of a tile sits at base + n * stride + l; in LDS at n * PC + l.
// Global accesses move V consecutive columns at once: V = 1 (one complex value, 8 bytes) or
// V = 2 (a 16-byte column pair; used where rows have an even pitch, so pairs are aligned and
// the partner of an odd last column is row padding, read and written but never used).
template <int V>
struct VecT;
template <>
struct VecT<1> {
  typedef float2 type;
  __device__ static float2 zero() { return make_float2(0.f, 0.f); }
};
template <>
struct VecT<2> {
  typedef float4 type;
  __device__ static float4 zero() { return make_float4(0.f, 0.f, 0.f, 0.f); }
};

template <int N, int PC, int NTH, int V>
__device__ __forceinline__ void load_tile(float2* lds, const float2* __restrict__ base,
                                          size_t stride, int ncols) {
  using T = typename VecT<V>::type;
  static_assert((N * PC) % (NTH * V) == 0, "whole tile per thread sweep");
#pragma unroll
  for (int m = 0; m < N * PC / (NTH * V); ++m) {
    const int p = threadIdx.x + m * NTH;
    const int n = p / (PC / V), l = (p % (PC / V)) * V;
    reinterpret_cast<T*>(lds)[p] =
        l < ncols ? *reinterpret_cast<const T*>(base + (size_t)n * stride + l) : VecT<V>::zero();
  }
}

// At 512^3 (spectra larger than the memory-side cache) the strided passes store with
// non-temporal writes, as the fused paints and the z passes do: the next pass reads the
// whole field back after it has been written (256^3/512^3 gradient 103.6 -> 101.1 ms).
template <int N, int PC, int NTH, int V>
__device__ __forceinline__ void store_tile(const float2* lds, float2* __restrict__ base,
                                           size_t stride, int ncols) {
  using T = typename VecT<V>::type;
  static_assert((N * PC) % (NTH * V) == 0, "whole tile per thread sweep");
#pragma unroll
  for (int m = 0; m < N * PC / (NTH * V); ++m) {
    const int p = threadIdx.x + m * NTH;
    const int n = p / (PC / V), l = (p % (PC / V)) * V;
    if (l < ncols) {
      if constexpr (N >= 512) {
#pragma unroll
        for (int u = 0; u < V; ++u)
          store_spec<true>(base + (size_t)n * stride + l + u, lds[p * V + u]);
      } else {
        *reinterpret_cast<T*>(base + (size_t)n * stride + l) = reinterpret_cast<const T*>(lds)[p];
      }
    }
  }
}

// Register image of a tile: thread t holds the units p = t + m * NTH (V columns each).
// Loading the next tile into registers while the current one is transformed overlaps the
// HBM latency with the LDS work.
template <int N, int PC, int NTH, int V>
struct TileRegs {
  static constexpr int PER = N * PC / (NTH * V);
  typename VecT<V>::type r[PER];
};

template <int N, int PC, int NTH, int V>
__device__ __forceinline__ void load_regs(TileRegs<N, PC, NTH, V>& t, const float2* __restrict__ base,
                                          size_t stride, int ncols) {
  using T = typename VecT<V>::type;
#pragma unroll
  for (int m = 0; m < TileRegs<N, PC, NTH, V>::PER; ++m) {
    const int p = threadIdx.x + m * NTH;
    const int n = p / (PC / V), l = (p % (PC / V)) * V;
    t.r[m] = l < ncols ? *reinterpret_cast<const T*>(base + (size_t)n * stride + l) : VecT<V>::zero();
  }
}

template <int N, int PC, int NTH, int V>
__device__ __forceinline__ void regs_to_lds(const TileRegs<N, PC, NTH, V>& t, float2* lds) {
  using T = typename VecT<V>::type;
#pragma unroll
  for (int m = 0; m < TileRegs<N, PC, NTH, V>::PER; ++m)
    reinterpret_cast<T*>(lds)[threadIdx.x + m * NTH] = t.r[m];
}

// y pass: in-place forward or inverse transform along y of each field. A workgroup walks
// the tiles blockIdx.x, blockIdx.x + gridDim.x, ... (tile = (field, x plane, kz chunk)),
// prefetching the next tile into registers.
template <int N, int DIR, int PC, int NTH, int V, int RMAX = 8>
__global__ __launch_bounds__(NTH) void ypass_kernel(float2* __restrict__ data, FieldMap m,
                                                    int ntiles, int ch0, int nchw) {
  constexpr int NH = N / 2 + 1;
  __shared__ __attribute__((aligned(16))) float2 lds[N * PC];
  __shared__ float2 tw[N];
  make_twiddles<N, NTH>(tw);
  auto tile_base = [&](int tau, int& ncols) {
    const int ch = ch0 + tau % nchw, rest = tau / nchw;
    const int ix = rest % N, f = rest / N;
    ncols = min(PC, NH - ch * PC);
    return data + m.off(f) + (size_t)ix * N * m.pitch + ch * PC;
  };
  int tau = xcd_block(blockIdx.x, gridDim.x);  // neighbouring tiles share an L2
  int nc;
  float2* b = tile_base(tau, nc);
  TileRegs<N, PC, NTH, V> pre;
  load_regs<N, PC, NTH, V>(pre, b, m.pitch, nc);
  for (;;) {
    regs_to_lds<N, PC, NTH, V>(pre, lds);
    __syncthreads();
    const int next = tau + gridDim.x;
    int nc2 = 0;
    float2* b2 = nullptr;
    if (next < ntiles) {
      b2 = tile_base(next, nc2);
      load_regs<N, PC, NTH, V>(pre, b2, m.pitch, nc2);
    }
    fft_lds<N, PC, PC, 1, 1, DIR, NTH, false, RMAX>(lds, tw);
    store_tile<N, PC, NTH, V>(lds, b, m.pitch, nc);
    if (next >= ntiles) break;
    __syncthreads();
    tau = next;
    b = b2;
    nc = nc2;
  }
}

// ---------------------------------------------------------------- x pass with operators
struct KVec {
  float kx, ky, kz, k2;
  int mx, my, mz;
};

template <int N>
__device__ __forceinline__ KVec kvec(int n, int iy, int kz, float kf) {
  KVec k;
  k.mx = wavenumber(n, N);
  k.my = wavenumber(iy, N);
  k.mz = kz;
  k.kx = kf * k.mx;
  k.ky = kf * k.my;
  k.kz = kf * k.mz;
  k.k2 = k.kx * k.kx + k.ky * k.ky + k.kz * k.kz;
  return k;
}

// i k_a / k^2 with the Nyquist plane of axis a and k = 0 removed; returned as the
// imaginary coefficient c (multiplier = i c). 1/k^2 from the hardware reciprocal (1 ulp).
template <int N>
__device__ __forceinline__ float grad_coef(const KVec& k, int a) {
  const int m = a == 0 ? k.mx : a == 1 ? k.my : k.mz;
  const float ka = a == 0 ? k.kx : a == 1 ? k.ky : k.kz;
  if (k.k2 == 0.f || m == N / 2 || m == -N / 2) return 0.f;
  return ka * __builtin_amdgcn_rcpf(k.k2);
}

// k_a k_b / k^2 (second derivative of the potential of the field, up to sign) with k = 0
// and the Nyquist planes of axes a and b removed, as each derivative in grad_coef.
template <int N>
__device__ __forceinline__ float hess_coef(const KVec& k, int a, int b) {
  const int ma = a == 0 ? k.mx : a == 1 ? k.my : k.mz;
  const int mb = b == 0 ? k.mx : b == 1 ? k.my : k.mz;
  const float ka = a == 0 ? k.kx : a == 1 ? k.ky : k.kz;
  const float kb = b == 0 ? k.kx : b == 1 ? k.ky : k.kz;
  if (k.k2 == 0.f || ma == N / 2 || ma == -N / 2 || mb == N / 2 || mb == -N / 2) return 0.f;
  return ka * kb * __builtin_amdgcn_rcpf(k.k2);
}

// 1 / k^2 with k = 0 removed (the potential of the split force operator).
template <int N>
__device__ __forceinline__ float inv_k2(const KVec& k) {
  return k.k2 == 0.f ? 0.f : __builtin_amdgcn_rcpf(k.k2);
}

// Pair o of a Hessian pair set: set 0 holds the diagonal (xx, yy, zz), set 1 the
// off-diagonal (xy, xz, yz).
__device__ __forceinline__ void hess_pair(int set, int o, int& a, int& b) {
  if (set == 0) {
    a = b = o;
  } else {
    a = o == 2 ? 1 : 0;
    b = o == 0 ? 1 : 2;
  }
}

template <int OP>
constexpr int xpass_inputs() {
  return (OP == XOP_FORCE_ADJ || OP == XOP_ZA_ADJ || OP == XOP_HESS_ADJ) ? 3
         : (OP == XOP_FEAT_ADJ || OP == XOP_FORCE_X_ADJ || OP == XOP_YGRAD_ADJ) ? 2
                                                                                  : 1;
}
template <int OP>
constexpr int xpass_outputs() {
  return (OP == XOP_FORCE || OP == XOP_ZA || OP == XOP_HESS) ? 3
         : (OP == XOP_GAUSS2 || OP == XOP_FORCE_X || OP == XOP_YGRAD) ? 2
                                                                      : 1;
}
// Operators whose input is already a full spectrum along the pass's axis (no forward
// transform along it).
template <int OP>
constexpr bool spectral_input() {
  return OP == XOP_ZA || OP == XOP_INV || OP == XOP_HESS || OP == XOP_YGRAD;
}
// Operators whose output is the forward transform itself (no inverse along the axis).
template <int OP>
constexpr bool spectral_output() {
  return OP == XOP_FWD || OP == XOP_YGRAD_ADJ;
}
// Operators on y lines: the line of a tile strides one row (pitch) instead of one plane
// (n rows), and the tile's fixed index is the x plane.
template <int OP>
constexpr bool yline() {
  return OP == XOP_YGRAD || OP == XOP_YGRAD_ADJ;
}

template <int N, int OP, int PC, int NTH, int V, int RMAX = 8>
__global__ __launch_bounds__(NTH) void xpass_kernel(XPassArgs a, int ntiles, int ch0, int nchw) {
  constexpr int NH = N / 2 + 1;
  constexpr int NE = N * PC;
  constexpr int PER = NE / NTH;
  static_assert(NE % NTH == 0, "tile");
  __shared__ __attribute__((aligned(16))) float2 lds[NE];
  __shared__ float2 tw[N];
  make_twiddles<N, NTH>(tw);
  constexpr bool YL = yline<OP>();
  // point stride along the transformed axis and the stride of the tile's fixed index
  const size_t istride = YL ? a.in_pitch : (size_t)N * a.in_pitch;
  const size_t ostride = YL ? a.out_pitch : (size_t)N * a.out_pitch;
  const size_t irow = YL ? (size_t)N * a.in_pitch : a.in_pitch;
  const size_t orow = YL ? (size_t)N * a.out_pitch : a.out_pitch;
  const size_t stride = (size_t)N * NH;  // prior table and projected modes (standard layout)
  const float kf = (float)(2.0 * M_PI / a.box);
  const float inv_n3 = (float)(1.0 / ((double)N * N * N));
  const int t = threadIdx.x;
  const int n_in = xpass_inputs<OP>();
  const int n_out = xpass_outputs<OP>();

  int tau = xcd_block(blockIdx.x, gridDim.x);  // neighbouring tiles share an L2
  TileRegs<N, PC, NTH, V> pre;  // the next input to transform (prefetched)
  {
    const int ch = ch0 + tau % nchw, iy = (tau / nchw) % N, item = tau / (nchw * N);
    const int kz0 = ch * PC;
    load_regs<N, PC, NTH, V>(pre, a.in[0] + item * a.in_item_stride + (size_t)iy * irow + kz0,
                          istride, min(PC, NH - kz0));
  }
  for (;;) {
    const int ch = ch0 + tau % nchw, iy = (tau / nchw) % N, item = tau / (nchw * N);
    const int kz0 = ch * PC;
    const int ncols = min(PC, NH - kz0);
    const size_t ioff = item * a.in_item_stride + (size_t)iy * irow + kz0;
    const size_t ooff = item * a.out_item_stride + (size_t)iy * orow + kz0;
    const int next = tau + gridDim.x;

    float2 hold[PER];  // spectrum (1-in ops) or accumulator (n-in ops)
#pragma unroll
    for (int m = 0; m < PER; ++m) hold[m] = make_float2(0.f, 0.f);
    float Rg = 0.f;
    if constexpr (OP == XOP_GAUSS) Rg = (float)a.params[item * NPRM + a.param_index];

    // -------- inputs (each prefetched into registers while the previous one is transformed:
    // the next input of this tile, after the last input the first input of the next tile)
    for (int i = 0; i < n_in; ++i) {
      regs_to_lds<N, PC, NTH, V>(pre, lds);
      __syncthreads();
      if (i + 1 < n_in) {
        load_regs<N, PC, NTH, V>(pre, a.in[i + 1] + ioff, istride, ncols);
      } else if (next < ntiles) {
        const int nch = ch0 + next % nchw, niy = (next / nchw) % N, nit = next / (nchw * N);
        const int nkz0 = nch * PC;
        load_regs<N, PC, NTH, V>(pre, a.in[0] + nit * a.in_item_stride + (size_t)niy * irow + nkz0,
                              istride, min(PC, NH - nkz0));
      }
      if constexpr (!spectral_input<OP>())
        fft_lds<N, PC, PC, 1, 1, -1, NTH, false, RMAX>(lds, tw);
#pragma unroll
      for (int m = 0; m < PER; ++m) {
        const int e = t + m * NTH;
        const int n = e / PC, l = e % PC;
        const float2 v = lds[e];
        if constexpr (OP == XOP_FORCE_ADJ || OP == XOP_ZA_ADJ) {
          const KVec k = kvec<N>(n, iy, kz0 + l, kf);
          const float c = grad_coef<N>(k, i);  // conj(i c) = -i c
          const float2 w = cmul_i<-1>(v);
          hold[m].x += c * w.x;
          hold[m].y += c * w.y;
        } else if constexpr (OP == XOP_FORCE_X_ADJ) {
          // conj(i k_x) A + B
          if (i == 0) {
            const float c = axis_coef<N>(n, kf);
            const float2 w = cmul_i<-1>(v);
            hold[m].x += c * w.x;
            hold[m].y += c * w.y;
          } else {
            hold[m].x += v.x;
            hold[m].y += v.y;
          }
        } else if constexpr (OP == XOP_YGRAD_ADJ) {
          // conj(i k_y) A + conj(i k_z) B
          const float c = i == 0 ? axis_coef<N>(n, kf) : axis_coef<N>(kz0 + l, kf);
          const float2 w = cmul_i<-1>(v);
          hold[m].x += c * w.x;
          hold[m].y += c * w.y;
        } else if constexpr (OP == XOP_HESS_ADJ) {
          const KVec k = kvec<N>(n, iy, kz0 + l, kf);
          int pa, pb;
          hess_pair(a.param_index, i, pa, pb);
          const float h = hess_coef<N>(k, pa, pb);  // real: its own conjugate
          hold[m].x += h * v.x;
          hold[m].y += h * v.y;
        } else if constexpr (OP == XOP_FEAT_ADJ) {
          const KVec k = kvec<N>(n, iy, kz0 + l, kf);
          const float g = i == 0 ? __expf(-0.5f * k.k2 * (float)(a.R1 * a.R1))
                                 : -__expf(-0.5f * k.k2 * (float)(a.R2 * a.R2));
          hold[m].x += g * v.x;
          hold[m].y += g * v.y;
        } else {
          hold[m] = v;
        }
      }
      __syncthreads();
    }

    // -------- outputs
    if constexpr (spectral_output<OP>()) {
#pragma unroll
      for (int m = 0; m < PER; ++m) lds[t + m * NTH] = hold[m];
      __syncthreads();
      store_tile<N, PC, NTH, V>(lds, a.out[0] + ooff, ostride, ncols);
    } else if constexpr (OP == XOP_ZA_ADJ) {
      // G = w(kz) (sum_a conj(M_a) g_a / n^3 + prior_weight loss_bar P s / S), G(0) = 0
      const double lam = a.params[item * NPRM + 5] * a.loss_bar[item];
#pragma unroll
      for (int m = 0; m < PER; ++m) {
        const int e = t + m * NTH;
        const int n = e / PC, l = e % PC;
        const int kz = kz0 + l;
        if (l >= ncols) continue;
        const size_t gi = (size_t)n * stride + (size_t)iy * NH + kz;
        const float wz = (kz == 0 || kz == N / 2) ? 1.f : 2.f;
        const float2 ps = a.proj_modes[item * a.aux_item_stride + gi];
        const float iv = a.inv_var[gi];
        float2 g = make_float2(hold[m].x * inv_n3 + (float)lam * iv * ps.x,
                               hold[m].y * inv_n3 + (float)lam * iv * ps.y);
        g.x *= wz;
        g.y *= wz;
        if (n == 0 && iy == 0 && kz == 0) g = make_float2(0.f, 0.f);
        a.out[0][item * a.out_item_stride + gi] = g;
      }
    } else if constexpr (OP == XOP_HESS_ADJ) {
      // G += w(kz) sum_ab h_ab g_ab / n^3, G(0) untouched (h vanishes there)
#pragma unroll
      for (int m = 0; m < PER; ++m) {
        const int e = t + m * NTH;
        const int n = e / PC, l = e % PC;
        const int kz = kz0 + l;
        if (l >= ncols) continue;
        const size_t gi = item * a.out_item_stride + (size_t)n * stride + (size_t)iy * NH + kz;
        const float wz = ((kz == 0 || kz == N / 2) ? 1.f : 2.f) * inv_n3;
        float2 g = a.out[0][gi];
        g.x += wz * hold[m].x;
        g.y += wz * hold[m].y;
        a.out[0][gi] = g;
      }
    } else {
      for (int o = 0; o < n_out; ++o) {
#pragma unroll
        for (int m = 0; m < PER; ++m) {
          const int e = t + m * NTH;
          const int n = e / PC, l = e % PC;
          float2 v = hold[m];
          if constexpr (OP == XOP_FORCE || OP == XOP_ZA) {
            const KVec k = kvec<N>(n, iy, kz0 + l, kf);
            const float c = grad_coef<N>(k, o) * inv_n3;
            v = cmul_i<1>(make_float2(c * v.x, c * v.y));
          } else if constexpr (OP == XOP_FORCE_X) {
            const KVec k = kvec<N>(n, iy, kz0 + l, kf);
            if (o == 0) {  // the x component
              const float c = grad_coef<N>(k, 0) * inv_n3;
              v = cmul_i<1>(make_float2(c * v.x, c * v.y));
            } else {  // the potential
              const float g = inv_k2<N>(k) * inv_n3;
              v = make_float2(g * v.x, g * v.y);
            }
          } else if constexpr (OP == XOP_FORCE_X_ADJ) {
            const KVec k = kvec<N>(n, iy, kz0 + l, kf);
            const float g = inv_k2<N>(k) * inv_n3;
            v = make_float2(g * v.x, g * v.y);
          } else if constexpr (OP == XOP_YGRAD) {  // i k_y A and i k_z A
            const float c = o == 0 ? axis_coef<N>(n, kf) : axis_coef<N>(kz0 + l, kf);
            v = cmul_i<1>(make_float2(c * v.x, c * v.y));
          } else if constexpr (OP == XOP_HESS) {
            const KVec k = kvec<N>(n, iy, kz0 + l, kf);
            int pa, pb;
            hess_pair(a.param_index, o, pa, pb);
            const float h = hess_coef<N>(k, pa, pb) * inv_n3;
            v = make_float2(h * v.x, h * v.y);
          } else if constexpr (OP == XOP_GAUSS) {
            const KVec k = kvec<N>(n, iy, kz0 + l, kf);
            const float g = __expf(-0.5f * k.k2 * Rg * Rg) * inv_n3;
            v = make_float2(g * v.x, g * v.y);
          } else if constexpr (OP == XOP_GAUSS2) {
            const KVec k = kvec<N>(n, iy, kz0 + l, kf);
            const float R = (float)(o == 0 ? a.R1 : a.R2);
            const float g = __expf(-0.5f * k.k2 * R * R) * inv_n3;
            v = make_float2(g * v.x, g * v.y);
          } else {  // XOP_INV, XOP_FORCE_ADJ, XOP_FEAT_ADJ
            v = make_float2(v.x * inv_n3, v.y * inv_n3);
          }
          lds[e] = v;
        }
        __syncthreads();
        fft_lds<N, PC, PC, 1, 1, +1, NTH, false, RMAX>(lds, tw);
        store_tile<N, PC, NTH, V>(lds, a.out[o] + ooff, ostride, ncols);
        __syncthreads();
      }
    }
    if (next >= ntiles) break;
    __syncthreads();
    tau = next;
  }
}

template <int N>
void zr2c(int fields, const float* in, FieldMap im, const float* in2, float a1, float a2,
          const double* sc, float2* out, FieldMap om, hipStream_t s) {
  dim3 grid((N * N) / ZTile<N>::ROWS, fields);
  zpass_r2c_kernel<N><<<grid, NT, 0, s>>>(in, im, in2, a1, a2, sc, out, om);
}

template <int N>
void zc2r3(int items, const float2* in, FieldMap im, Vec3* out, size_t out_item_stride,
           hipStream_t s) {
  const int per = (N * N) / ZTile3<N>::R, ntiles = per * items;
  const int res = resident_grid<zpass_c2r3_kernel<N>, NT>();
  zpass_c2r3_kernel<N><<<ntiles < res ? ntiles : res, NT, 0, s>>>(
      in, im, out, out_item_stride, per, ntiles);
}

template <int N>
void zc2r(int fields, const float2* in, FieldMap im, float* out, FieldMap om, const float* add,
          hipStream_t s) {
  const int per = (N * N) / ZTile<N>::ROWS, ntiles = per * fields;
  const int res = resident_grid<zpass_c2r_kernel<N>, NT>();
  zpass_c2r_kernel<N><<<ntiles < res ? ntiles : res, NT, 0, s>>>(
      in, im, out, om, add, per, ntiles);
}

int log2i(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

// ---------------------------------------------------------------- register-resident passes
// Each thread keeps P = N * PC / NTH points of its lines in registers across a whole
// transform. A stage with radix R works on P / R butterflies per thread, slot j of thread t
// being butterfly b = t + j * NTH (line l = b % PC, index i = b / PC). The first stage
// reads its inputs straight from HBM and the last stage writes straight to HBM; LDS is
// used only for the permutations between stages. The inverse runs the radices in reverse
// order, so the forward's output registers are exactly the inverse's input registers and a
// k-space operator sits between them with no data movement.
template <int N, bool REV>
struct RPlan {
  static constexpr int S8 = N >= 512 ? 3 : N >= 64 ? 2 : N >= 8 ? 1 : 0;
  static constexpr int P8 = S8 == 3 ? 512 : S8 == 2 ? 64 : S8 == 1 ? 8 : 1;
  static constexpr int REM = N / P8;  // 1, 2 or 4
  static constexpr int S = S8 + (REM > 1 ? 1 : 0);
  static constexpr int radix(int s) {
    return REV ? ((REM > 1 && s == 0) ? REM : 8) : (s < S8 ? 8 : REM);
  }
  static constexpr int prev(int s) {
    int p = 1;
    for (int q = 0; q < s; ++q) p *= radix(q);
    return p;
  }
};

template <int N, int PC, int NTH>
constexpr bool reg_ok() {
  return (N * PC) % NTH == 0 && (N * PC / NTH) >= 8 && ((N * PC / NTH) % 8) == 0 && N >= 64;
}

// Butterflies of one stage, in registers (twiddles for PREV > 1 from the table tw[], which
// holds exp(-2 pi i j / N), j < N).
template <int N, int PC, int NTH, int R, int PREV, int DIR>
__device__ __forceinline__ void reg_stage(float2* v, const float2* tw) {
  constexpr int P = N * PC / NTH;
#pragma unroll
  for (int j = 0; j < P / R; ++j) {
    float2* u = v + j * R;
    if constexpr (PREV > 1) {
      const int i = (threadIdx.x + j * NTH) / PC;
      const int k = i & (PREV - 1);
#pragma unroll
      for (int r = 1; r < R; ++r) {
        float2 w = tw[r * k * (N / (PREV * R))];
        if (DIR > 0) w.y = -w.y;
        u[r] = cmul(u[r], w);
      }
    }
    bfly<R, DIR>(u);
  }
}

// Permutation from the outputs of stage (R, PREV) to the inputs of stage (R2) through LDS.
template <int N, int PC, int NTH, int R, int PREV, int R2>
__device__ __forceinline__ void reg_exchange(float2* v, float2* lds) {
  constexpr int P = N * PC / NTH;
#pragma unroll
  for (int j = 0; j < P / R; ++j) {
    const int b = threadIdx.x + j * NTH;
    const int i = b / PC, l = b % PC;
    const int k = i & (PREV - 1);
    const int j0 = (i - k) * R + k;
#pragma unroll
    for (int r = 0; r < R; ++r) lds[(j0 + r * PREV) * PC + l] = v[j * R + r];
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < P / R2; ++j) {
    const int b = threadIdx.x + j * NTH;
    const int i = b / PC, l = b % PC;
#pragma unroll
    for (int r = 0; r < R2; ++r) v[j * R2 + r] = lds[(i + r * (N / R2)) * PC + l];
  }
  __syncthreads();
}

template <int N, int PC, int NTH, bool REV, int DIR, int S>
__device__ __forceinline__ void reg_stages_from(float2* v, float2* lds, const float2* tw) {
  using PL = RPlan<N, REV>;
  if constexpr (S < PL::S) {
    constexpr int R = PL::radix(S), PV = PL::prev(S);
    reg_stage<N, PC, NTH, R, PV, DIR>(v, tw);
    if constexpr (S + 1 < PL::S) {
      reg_exchange<N, PC, NTH, R, PV, PL::radix(S + 1)>(v, lds);
      reg_stages_from<N, PC, NTH, REV, DIR, S + 1>(v, lds, tw);
    }
  }
}

// Whole transform of the thread's lines: v holds the inputs in the first stage's slot order
// and returns the outputs in the last stage's slot order.
template <int N, int PC, int NTH, bool REV, int DIR>
__device__ __forceinline__ void reg_fft(float2* v, float2* lds, const float2* tw) {
  reg_stages_from<N, PC, NTH, REV, DIR, 0>(v, lds, tw);
}

// HBM <-> registers in first-stage order (inputs at i + r N/R) or last-stage order (outputs
// at i + r N/R of the last radix R, since the last stage has PREV = N/R).
template <int N, int PC, int NTH, int R>
__device__ __forceinline__ void reg_load(float2* v, const float2* __restrict__ base,
                                         size_t stride, int ncols) {
  constexpr int P = N * PC / NTH;
#pragma unroll
  for (int j = 0; j < P / R; ++j) {
    const int b = threadIdx.x + j * NTH;
    const int i = b / PC, l = b % PC;
#pragma unroll
    for (int r = 0; r < R; ++r)
      v[j * R + r] = l < ncols ? base[(size_t)(i + r * (N / R)) * stride + l] : make_float2(0.f, 0.f);
  }
}

template <int N, int PC, int NTH, int R>
__device__ __forceinline__ void reg_store(const float2* v, float2* __restrict__ base, size_t stride,
                                          int ncols) {
  constexpr int P = N * PC / NTH;
#pragma unroll
  for (int j = 0; j < P / R; ++j) {
    const int b = threadIdx.x + j * NTH;
    const int i = b / PC, l = b % PC;
    if (l < ncols) {
#pragma unroll
      for (int r = 0; r < R; ++r)
        store_spec<(N >= 512)>(&base[(size_t)(i + r * (N / R)) * stride + l], v[j * R + r]);
    }
  }
}

// Point index (along the transformed axis) and line of register slot q in last-stage order.
template <int N, int PC, int NTH, int R>
__device__ __forceinline__ void reg_slot(int q, int& pos, int& l) {
  const int j = q / R, r = q % R;
  const int b = threadIdx.x + j * NTH;
  l = b % PC;
  pos = b / PC + r * (N / R);
}

template <int N, int DIR, int PC, int NTH>
__global__ __launch_bounds__(NTH) void ypass_reg_kernel(float2* __restrict__ data, FieldMap m,
                                                        int ntiles, int ch0, int nchw) {
  constexpr int NH = N / 2 + 1;
  constexpr int P = N * PC / NTH;
  constexpr bool REV = DIR > 0;
  using PL = RPlan<N, REV>;
  constexpr int R0 = PL::radix(0), RL = PL::radix(PL::S - 1);
  __shared__ float2 lds[N * PC];
  __shared__ float2 tw[N];
  make_twiddles<N, NTH>(tw);
  auto tile_base = [&](int tau, int& ncols) {
    const int ch = ch0 + tau % nchw, rest = tau / nchw;
    const int ix = rest % N, f = rest / N;
    ncols = min(PC, NH - ch * PC);
    return data + m.off(f) + (size_t)ix * N * m.pitch + ch * PC;
  };
  int tau = xcd_block(blockIdx.x, gridDim.x);  // neighbouring tiles share an L2
  int nc;
  float2* b = tile_base(tau, nc);
  float2 pre[P], v[P];
  reg_load<N, PC, NTH, R0>(pre, b, m.pitch, nc);
  __syncthreads();  // twiddles
  for (;;) {
#pragma unroll
    for (int q = 0; q < P; ++q) v[q] = pre[q];
    const int next = tau + gridDim.x;
    int nc2 = 0;
    float2* b2 = nullptr;
    if (next < ntiles) {
      b2 = tile_base(next, nc2);
      reg_load<N, PC, NTH, R0>(pre, b2, m.pitch, nc2);
    }
    reg_fft<N, PC, NTH, REV, DIR>(v, lds, tw);
    reg_store<N, PC, NTH, RL>(v, b, m.pitch, nc);
    if (next >= ntiles) break;
    tau = next;
    b = b2;
    nc = nc2;
  }
}

template <int N, int OP, int PC, int NTH>
__global__ __launch_bounds__(NTH) void xpass_reg_kernel(XPassArgs a, int ntiles, int ch0,
                                                        int nchw) {
  constexpr int NH = N / 2 + 1;
  constexpr int P = N * PC / NTH;
  using PF = RPlan<N, false>;
  using PI = RPlan<N, true>;
  constexpr int R0F = PF::radix(0), RLF = PF::radix(PF::S - 1);
  constexpr int RLI = PI::radix(PI::S - 1);
  static_assert(PI::radix(0) == RLF, "inverse starts with the forward's last radix");
  constexpr bool SPECTRAL_IN = spectral_input<OP>();
  constexpr int RIN = SPECTRAL_IN ? RLF : R0F;  // layout in which inputs are loaded
  __shared__ float2 lds[N * PC];
  __shared__ float2 tw[N];
  make_twiddles<N, NTH>(tw);
  constexpr bool YL = yline<OP>();
  // point stride along the transformed axis and the stride of the tile's fixed index
  const size_t istride = YL ? a.in_pitch : (size_t)N * a.in_pitch;
  const size_t ostride = YL ? a.out_pitch : (size_t)N * a.out_pitch;
  const size_t irow = YL ? (size_t)N * a.in_pitch : a.in_pitch;
  const size_t orow = YL ? (size_t)N * a.out_pitch : a.out_pitch;
  const size_t stride = (size_t)N * NH;  // prior table, projected modes, gradient
  const float kf = (float)(2.0 * M_PI / a.box);
  const float inv_n3 = (float)(1.0 / ((double)N * N * N));
  constexpr int n_in = xpass_inputs<OP>();
  constexpr int n_out = xpass_outputs<OP>();

  auto in_base = [&](int tau, int i, int& ncols) {
    const int ch = ch0 + tau % nchw, iy = (tau / nchw) % N, item = tau / (nchw * N);
    ncols = min(PC, NH - ch * PC);
    return a.in[i] + item * a.in_item_stride + (size_t)iy * irow + ch * PC;
  };
  int tau = xcd_block(blockIdx.x, gridDim.x);  // neighbouring tiles share an L2
  float2 pre[P];
  {
    int nc;
    const float2* b0 = in_base(tau, 0, nc);
    reg_load<N, PC, NTH, RIN>(pre, b0, istride, nc);
  }
  __syncthreads();  // twiddles
  for (;;) {
    const int ch = ch0 + tau % nchw, iy = (tau / nchw) % N, item = tau / (nchw * N);
    const int kz0 = ch * PC;
    const int ncols = min(PC, NH - kz0);
    const size_t ooff = item * a.out_item_stride + (size_t)iy * orow + kz0;
    const int next = tau + gridDim.x;
    float Rg = 0.f;
    if constexpr (OP == XOP_GAUSS) Rg = (float)a.params[item * NPRM + a.param_index];

    float2 hold[P];
#pragma unroll
    for (int q = 0; q < P; ++q) hold[q] = make_float2(0.f, 0.f);
    // -------- inputs (each prefetched while the previous one is transformed)
#pragma unroll 1
    for (int i = 0; i < n_in; ++i) {
      float2 v[P];
#pragma unroll
      for (int q = 0; q < P; ++q) v[q] = pre[q];
      if (i + 1 < n_in) {
        int nc;
        const float2* bi = in_base(tau, i + 1, nc);
        reg_load<N, PC, NTH, RIN>(pre, bi, istride, nc);
      } else if (next < ntiles) {
        int nc;
        const float2* bn = in_base(next, 0, nc);
        reg_load<N, PC, NTH, RIN>(pre, bn, istride, nc);
      }
      if constexpr (!SPECTRAL_IN) reg_fft<N, PC, NTH, false, -1>(v, lds, tw);
#pragma unroll
      for (int q = 0; q < P; ++q) {
        if constexpr (OP == XOP_FORCE_ADJ || OP == XOP_ZA_ADJ) {
          int n, l;
          reg_slot<N, PC, NTH, RLF>(q, n, l);
          const KVec k = kvec<N>(n, iy, kz0 + l, kf);
          const float c = grad_coef<N>(k, i);  // conj(i c) = -i c
          const float2 w = cmul_i<-1>(v[q]);
          hold[q].x += c * w.x;
          hold[q].y += c * w.y;
        } else if constexpr (OP == XOP_FORCE_X_ADJ) {
          // conj(i k_x) A + B
          if (i == 0) {
            int n, l;
            reg_slot<N, PC, NTH, RLF>(q, n, l);
            const float c = axis_coef<N>(n, kf);
            const float2 w = cmul_i<-1>(v[q]);
            hold[q].x += c * w.x;
            hold[q].y += c * w.y;
          } else {
            hold[q].x += v[q].x;
            hold[q].y += v[q].y;
          }
        } else if constexpr (OP == XOP_YGRAD_ADJ) {
          // conj(i k_y) A + conj(i k_z) B
          int n, l;
          reg_slot<N, PC, NTH, RLF>(q, n, l);
          const float c = i == 0 ? axis_coef<N>(n, kf) : axis_coef<N>(kz0 + l, kf);
          const float2 w = cmul_i<-1>(v[q]);
          hold[q].x += c * w.x;
          hold[q].y += c * w.y;
        } else if constexpr (OP == XOP_HESS_ADJ) {
          int n, l;
          reg_slot<N, PC, NTH, RLF>(q, n, l);
          const KVec k = kvec<N>(n, iy, kz0 + l, kf);
          int pa, pb;
          hess_pair(a.param_index, i, pa, pb);
          const float h = hess_coef<N>(k, pa, pb);  // real: its own conjugate
          hold[q].x += h * v[q].x;
          hold[q].y += h * v[q].y;
        } else if constexpr (OP == XOP_FEAT_ADJ) {
          int n, l;
          reg_slot<N, PC, NTH, RLF>(q, n, l);
          const KVec k = kvec<N>(n, iy, kz0 + l, kf);
          const float g = i == 0 ? __expf(-0.5f * k.k2 * (float)(a.R1 * a.R1))
                                 : -__expf(-0.5f * k.k2 * (float)(a.R2 * a.R2));
          hold[q].x += g * v[q].x;
          hold[q].y += g * v[q].y;
        } else {
          hold[q] = v[q];
        }
      }
    }
    // -------- outputs
    if constexpr (spectral_output<OP>()) {
      reg_store<N, PC, NTH, RLF>(hold, a.out[0] + ooff, ostride, ncols);
    } else if constexpr (OP == XOP_ZA_ADJ) {
      // G = w(kz) (sum_a conj(M_a) g_a / n^3 + prior_weight loss_bar P s / S), G(0) = 0
      const double lam = a.params[item * NPRM + 5] * a.loss_bar[item];
#pragma unroll
      for (int q = 0; q < P; ++q) {
        int n, l;
        reg_slot<N, PC, NTH, RLF>(q, n, l);
        const int kz = kz0 + l;
        if (l >= ncols) continue;
        const size_t gi = (size_t)n * stride + (size_t)iy * NH + kz;
        const float wz = (kz == 0 || kz == N / 2) ? 1.f : 2.f;
        const float2 ps = a.proj_modes[item * a.aux_item_stride + gi];
        const float iv = a.inv_var[gi];
        float2 g = make_float2(hold[q].x * inv_n3 + (float)lam * iv * ps.x,
                               hold[q].y * inv_n3 + (float)lam * iv * ps.y);
        g.x *= wz;
        g.y *= wz;
        if (n == 0 && iy == 0 && kz == 0) g = make_float2(0.f, 0.f);
        a.out[0][item * a.out_item_stride + gi] = g;
      }
    } else if constexpr (OP == XOP_HESS_ADJ) {
      // G += w(kz) sum_ab h_ab g_ab / n^3, G(0) untouched (h vanishes there)
#pragma unroll
      for (int q = 0; q < P; ++q) {
        int n, l;
        reg_slot<N, PC, NTH, RLF>(q, n, l);
        const int kz = kz0 + l;
        if (l >= ncols) continue;
        const size_t gi = item * a.out_item_stride + (size_t)n * stride + (size_t)iy * NH + kz;
        const float wz = ((kz == 0 || kz == N / 2) ? 1.f : 2.f) * inv_n3;
        float2 g = a.out[0][gi];
        g.x += wz * hold[q].x;
        g.y += wz * hold[q].y;
        a.out[0][gi] = g;
      }
    } else {
#pragma unroll
      for (int o = 0; o < n_out; ++o) {
        float2 v[P];
#pragma unroll
        for (int q = 0; q < P; ++q) {
          int n, l;
          reg_slot<N, PC, NTH, RLF>(q, n, l);
          float2 x = hold[q];
          if constexpr (OP == XOP_FORCE || OP == XOP_ZA) {
            const KVec k = kvec<N>(n, iy, kz0 + l, kf);
            const float c = grad_coef<N>(k, o) * inv_n3;
            x = cmul_i<1>(make_float2(c * x.x, c * x.y));
          } else if constexpr (OP == XOP_FORCE_X) {
            const KVec k = kvec<N>(n, iy, kz0 + l, kf);
            if (o == 0) {  // the x component
              const float c = grad_coef<N>(k, 0) * inv_n3;
              x = cmul_i<1>(make_float2(c * x.x, c * x.y));
            } else {  // the potential
              const float g = inv_k2<N>(k) * inv_n3;
              x = make_float2(g * x.x, g * x.y);
            }
          } else if constexpr (OP == XOP_FORCE_X_ADJ) {
            const KVec k = kvec<N>(n, iy, kz0 + l, kf);
            const float g = inv_k2<N>(k) * inv_n3;
            x = make_float2(g * x.x, g * x.y);
          } else if constexpr (OP == XOP_YGRAD) {  // i k_y A and i k_z A
            const float c = o == 0 ? axis_coef<N>(n, kf) : axis_coef<N>(kz0 + l, kf);
            x = cmul_i<1>(make_float2(c * x.x, c * x.y));
          } else if constexpr (OP == XOP_HESS) {
            const KVec k = kvec<N>(n, iy, kz0 + l, kf);
            int pa, pb;
            hess_pair(a.param_index, o, pa, pb);
            const float h = hess_coef<N>(k, pa, pb) * inv_n3;
            x = make_float2(h * x.x, h * x.y);
          } else if constexpr (OP == XOP_GAUSS) {
            const KVec k = kvec<N>(n, iy, kz0 + l, kf);
            const float g = __expf(-0.5f * k.k2 * Rg * Rg) * inv_n3;
            x = make_float2(g * x.x, g * x.y);
          } else if constexpr (OP == XOP_GAUSS2) {
            const KVec k = kvec<N>(n, iy, kz0 + l, kf);
            const float R = (float)(o == 0 ? a.R1 : a.R2);
            const float g = __expf(-0.5f * k.k2 * R * R) * inv_n3;
            x = make_float2(g * x.x, g * x.y);
          } else {  // XOP_INV, XOP_FORCE_ADJ, XOP_FEAT_ADJ
            x = make_float2(x.x * inv_n3, x.y * inv_n3);
          }
          v[q] = x;
        }
        reg_fft<N, PC, NTH, true, +1>(v, lds, tw);
        reg_store<N, PC, NTH, RLI>(v, a.out[o] + ooff, ostride, ncols);
      }
    }
    if (next >= ntiles) break;
    tau = next;
  }
}

// 16-byte column pairs need an even number of elements per thread.
template <int N, int PC, int NTH>
constexpr bool pairs_ok() {
  return (N * PC) % (2 * NTH) == 0;
}

// Tile loops launch the resident number of workgroups (at most the number of tiles).
template <auto Kernel, int NTH>
int tile_grid(int ntiles) {
  const int res = resident_grid<Kernel, NTH>();
  return ntiles < res ? ntiles : res;
}

// Chunks [ch0, ch0 + nchw) of PC columns covering the kz window [lo, hi) (hi = 0: the whole
// half spectrum); lo is a multiple of PC (the caller picks windows on multiples of every
// pass's column count).
template <int N, int PC>
__host__ inline void kz_chunks(int lo, int hi, int& ch0, int& nchw) {
  constexpr int NH = N / 2 + 1;
  const int h = (hi > 0 && hi < NH) ? hi : NH;
  ch0 = lo / PC;
  nchw = (h + PC - 1) / PC - ch0;
}

// Staging of the strided passes: 0 register-resident (radix-8 plan), 1 LDS-staged radix-8
// plan, 2 LDS-staged radix-4 plan.
template <int N, int DIR, int PC, int NTH, int V>
void ypass_lds_launch(int staging, float2* d, FieldMap m, int ntiles, int ch0, int nchw,
                      hipStream_t s) {
  if (staging == 2) {
    constexpr auto k = ypass_kernel<N, DIR, PC, NTH, V, 4>;
    k<<<tile_grid<k, NTH>(ntiles), NTH, 0, s>>>(d, m, ntiles, ch0, nchw);
  } else {
    constexpr auto k = ypass_kernel<N, DIR, PC, NTH, V, 8>;
    k<<<tile_grid<k, NTH>(ntiles), NTH, 0, s>>>(d, m, ntiles, ch0, nchw);
  }
}

template <int N, int PC, int NTH>
void ypass_t(int fields, float2* d, FieldMap m, bool inv, int staging, hipStream_t s,
             KzWin win) {
  int ch0, nchw;
  kz_chunks<N, PC>(win.lo, win.hi, ch0, nchw);
  if (nchw <= 0) return;
  const int ntiles = nchw * N * fields;
  if constexpr (reg_ok<N, PC, NTH>()) {
    if (staging == 0) {
      if (inv) {
        constexpr auto k = ypass_reg_kernel<N, +1, PC, NTH>;
        k<<<tile_grid<k, NTH>(ntiles), NTH, 0, s>>>(d, m, ntiles, ch0, nchw);
      } else {
        constexpr auto k = ypass_reg_kernel<N, -1, PC, NTH>;
        k<<<tile_grid<k, NTH>(ntiles), NTH, 0, s>>>(d, m, ntiles, ch0, nchw);
      }
      return;
    }
  }
  if constexpr (pairs_ok<N, PC, NTH>()) {
    if (m.pitch % 2 == 0) {
      if (inv)
        ypass_lds_launch<N, +1, PC, NTH, 2>(staging, d, m, ntiles, ch0, nchw, s);
      else
        ypass_lds_launch<N, -1, PC, NTH, 2>(staging, d, m, ntiles, ch0, nchw, s);
      return;
    }
  }
  if (inv)
    ypass_lds_launch<N, +1, PC, NTH, 1>(staging, d, m, ntiles, ch0, nchw, s);
  else
    ypass_lds_launch<N, -1, PC, NTH, 1>(staging, d, m, ntiles, ch0, nchw, s);
}

template <int N, int OP, int PC, int NTH, int V>
void xpass_lds_launch(int staging, const XPassArgs& a, int ntiles, int ch0, int nchw,
                      hipStream_t s) {
  if (staging == 2) {
    constexpr auto k = xpass_kernel<N, OP, PC, NTH, V, 4>;
    k<<<tile_grid<k, NTH>(ntiles), NTH, 0, s>>>(a, ntiles, ch0, nchw);
  } else {
    constexpr auto k = xpass_kernel<N, OP, PC, NTH, V, 8>;
    k<<<tile_grid<k, NTH>(ntiles), NTH, 0, s>>>(a, ntiles, ch0, nchw);
  }
}

template <int N, int OP, int PC, int NTH>
void xpass_t(const XPassArgs& a, int staging, hipStream_t s) {
  int ch0, nchw;
  kz_chunks<N, PC>(a.kz_lo, a.kz_hi, ch0, nchw);
  if (nchw <= 0) return;
  const int ntiles = nchw * N * a.batch;
  if constexpr (reg_ok<N, PC, NTH>()) {
    if (staging == 0) {
      constexpr auto k = xpass_reg_kernel<N, OP, PC, NTH>;
      k<<<tile_grid<k, NTH>(ntiles), NTH, 0, s>>>(a, ntiles, ch0, nchw);
      return;
    }
  }
  if constexpr (pairs_ok<N, PC, NTH>() && OP != XOP_ZA && OP != XOP_ZA_ADJ && OP != XOP_HESS &&
                OP != XOP_HESS_ADJ) {
    if (a.in_pitch % 2 == 0 && a.out_pitch % 2 == 0) {
      xpass_lds_launch<N, OP, PC, NTH, 2>(staging, a, ntiles, ch0, nchw, s);
      return;
    }
  }
  xpass_lds_launch<N, OP, PC, NTH, 1>(staging, a, ntiles, ch0, nchw, s);
}

// Supported shapes: PC in {8, 16, 32}, NTH in {256, 512}, with N * PC >= NTH and the LDS
// tile N * PC * 8 B + N * 8 B within 160 KB.
template <int N>
constexpr bool shape_ok(int pc, int nth) {
  return N * pc >= nth && (N * pc + N) * 8 <= 160 * 1024 && N * pc / nth <= 16;
}

#define PMR_FOR_SHAPE(M) M(8, 256) M(16, 256) M(32, 256) M(8, 512) M(16, 512) M(32, 512)

template <int N>
void ypass(int fields, float2* d, FieldMap m, bool inv, hipStream_t s, KzWin win) {
  const TileShape t = g_fft_tile[0][log2i(N)];
#define SHAPE(PC, NTH)                                        \
  if constexpr (shape_ok<N>(PC, NTH))                         \
    if (t.pc == PC && t.nth == NTH) {                         \
      ypass_t<N, PC, NTH>(fields, d, m, inv, t.staging, s, win);  \
      return;                                                     \
    }
  PMR_FOR_SHAPE(SHAPE)
#undef SHAPE
  ypass_t<N, 16, 256>(fields, d, m, inv, t.staging, s, win);
}

// Multi-input operators hold three register images (accumulator, current, prefetch); at
// more than 8 points per thread they would spill, so they run on half-width tiles.
template <int OP>
constexpr bool multi_input() {
  return OP == XOP_FORCE_ADJ || OP == XOP_FEAT_ADJ || OP == XOP_ZA_ADJ || OP == XOP_HESS_ADJ ||
         OP == XOP_FORCE_X_ADJ || OP == XOP_YGRAD_ADJ;
}

template <int N, int OP>
void xpass_op(const XPassArgs& a, hipStream_t s) {
  const TileShape t = g_fft_tile[multi_input<OP>() ? 2 : 1][log2i(N)];
#define SHAPE(PC, NTH)                                                         \
  if constexpr (shape_ok<N>(PC, NTH))                                          \
    if (t.pc == PC && t.nth == NTH) {                                          \
      if constexpr (multi_input<OP>() && N * PC / NTH > 8 && PC > 8)           \
        if (t.staging == 0) {                                                  \
          xpass_t<N, OP, PC / 2, NTH>(a, 0, s);                                \
          return;                                                              \
        }                                                                      \
      xpass_t<N, OP, PC, NTH>(a, t.staging, s);                                \
      return;                                                                  \
    }
  PMR_FOR_SHAPE(SHAPE)
#undef SHAPE
  xpass_t<N, OP, 16, 256>(a, t.staging, s);
}

template <int N>
void xpass_dispatch(int op, const XPassArgs& a, hipStream_t s) {
  switch (op) {
    case XOP_FWD: xpass_op<N, XOP_FWD>(a, s); break;
    case XOP_INV: xpass_op<N, XOP_INV>(a, s); break;
    case XOP_FORCE: xpass_op<N, XOP_FORCE>(a, s); break;
    case XOP_FORCE_ADJ: xpass_op<N, XOP_FORCE_ADJ>(a, s); break;
    case XOP_GAUSS: xpass_op<N, XOP_GAUSS>(a, s); break;
    case XOP_GAUSS2: xpass_op<N, XOP_GAUSS2>(a, s); break;
    case XOP_FEAT_ADJ: xpass_op<N, XOP_FEAT_ADJ>(a, s); break;
    case XOP_ZA: xpass_op<N, XOP_ZA>(a, s); break;
    case XOP_ZA_ADJ: xpass_op<N, XOP_ZA_ADJ>(a, s); break;
    case XOP_HESS: xpass_op<N, XOP_HESS>(a, s); break;
    case XOP_HESS_ADJ: xpass_op<N, XOP_HESS_ADJ>(a, s); break;
    case XOP_FORCE_X: xpass_op<N, XOP_FORCE_X>(a, s); break;
    case XOP_FORCE_X_ADJ: xpass_op<N, XOP_FORCE_X_ADJ>(a, s); break;
    case XOP_YGRAD: xpass_op<N, XOP_YGRAD>(a, s); break;
    case XOP_YGRAD_ADJ: xpass_op<N, XOP_YGRAD_ADJ>(a, s); break;
    default: break;
  }
}

}  // namespace
}  // namespace pmr
