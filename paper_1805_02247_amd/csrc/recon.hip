// Reconstruction driver support (Sec. 5.2, Sec. 5.3): the vector algebra of L-BFGS over the
// linear modes with FP64 inner products and device-resident scalars, and the binned
// two-point statistics that score a reconstruction (Sec. 4.3).
//
// Inner products: each element product is exact in FP64 (two FP32 factors), the partial
// sums of a fixed grid and the final tree are fixed, so results are bitwise reproducible.
#include "../../include/pmr.h"

#include <mutex>

#include "pmr_internal.h"

namespace pmr {
namespace {

constexpr int TB = 256;
constexpr int DOT_BLOCKS = 1024;  // partial sums per inner product (at most)

__device__ __forceinline__ double block_sum(double v, double* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int d = TB / 2; d > 0; d >>= 1) {
    if (t < d) sh[t] += sh[t + d];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

int dot_blocks(size_t n) {
  const size_t b = (n + (size_t)TB * 8 - 1) / ((size_t)TB * 8);
  return (int)(b < 1 ? 1 : b > DOT_BLOCKS ? DOT_BLOCKS : b);
}

// partial[block] = sum over this block's grid-stride elements of a[i] b[i] (FP64).
__global__ __launch_bounds__(TB) void dot_partial_kernel(const float* __restrict__ a,
                                                         const float* __restrict__ b, size_t n,
                                                         double* __restrict__ partial) {
  __shared__ double sh[TB];
  double acc = 0.0;
  const size_t stride = (size_t)gridDim.x * TB;
  for (size_t i = (size_t)blockIdx.x * TB + threadIdx.x; i < n; i += stride)
    acc += (double)a[i] * (double)b[i];
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// out = (sum of the partials) / den (den: device scalar, or 1).
__global__ __launch_bounds__(TB) void dot_final_kernel(const double* __restrict__ partial, int np,
                                                       const double* __restrict__ den,
                                                       double* __restrict__ out) {
  __shared__ double sh[TB];
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += TB) acc += partial[i];
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) out[0] = den ? s / den[0] : s;
}

// y += sign * (A - B) * x with A, B device scalars (B nullable).
__global__ __launch_bounds__(TB) void axpy_dev_kernel(size_t n, const double* __restrict__ A,
                                                      const double* __restrict__ B, double sign,
                                                      const float* __restrict__ x,
                                                      float* __restrict__ y) {
  const float c = (float)(sign * (A[0] - (B ? B[0] : 0.0)));
  const size_t stride = (size_t)gridDim.x * TB;
  for (size_t i = (size_t)blockIdx.x * TB + threadIdx.x; i < n; i += stride) y[i] += c * x[i];
}

// x *= sign * num / den (device scalars).
__global__ __launch_bounds__(TB) void scale_dev_kernel(size_t n, const double* __restrict__ num,
                                                       const double* __restrict__ den, double sign,
                                                       float* __restrict__ x) {
  const float c = (float)(sign * num[0] / den[0]);
  const size_t stride = (size_t)gridDim.x * TB;
  for (size_t i = (size_t)blockIdx.x * TB + threadIdx.x; i < n; i += stride) x[i] *= c;
}

// out = alpha a + beta b (host scalars; out may alias a or b).
__global__ __launch_bounds__(TB) void axpby_kernel(size_t n, float alpha, const float* a,
                                                   float beta, const float* b, float* out) {
  const size_t stride = (size_t)gridDim.x * TB;
  for (size_t i = (size_t)blockIdx.x * TB + threadIdx.x; i < n; i += stride)
    out[i] = alpha * a[i] + beta * b[i];
}

unsigned stream_grid(size_t n) {
  const size_t b = (n + TB - 1) / TB;
  return (unsigned)(b > 4096 ? 4096 : b < 1 ? 1 : b);
}

// ---------------------------------------------------------------- binned spectra
constexpr int PS_THREADS = 2048;  // accumulating threads (each owns a contiguous mode range)

// Thread t accumulates modes [t chunk, (t + 1) chunk) of the half spectrum into its own
// slice work[q][bin][t] (q = count, |a|^2, |b|^2, Re a conj b; Hermitian weight applied),
// flushing its running sums whenever the shell changes (consecutive kz rarely change it).
__global__ __launch_bounds__(TB) void power_partial_kernel(int n, const float2* __restrict__ a,
                                                           const float2* __restrict__ b,
                                                           int nbins, size_t chunk,
                                                           double* __restrict__ work) {
  const int t = blockIdx.x * TB + threadIdx.x;
  if (t >= PS_THREADS) return;
  const int h = n / 2 + 1;
  const size_t total = (size_t)n * n * h;
  for (int q = 0; q < 4; ++q)
    for (int k = 0; k < nbins; ++k) work[((size_t)q * nbins + k) * PS_THREADS + t] = 0.0;
  const size_t lo = (size_t)t * chunk;
  const size_t hi = lo + chunk < total ? lo + chunk : total;
  int cur = -1;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  auto flush = [&]() {
    if (cur >= 0)
      for (int q = 0; q < 4; ++q) work[((size_t)q * nbins + cur) * PS_THREADS + t] += acc[q];
    acc[0] = acc[1] = acc[2] = acc[3] = 0.0;
  };
  for (size_t e = lo; e < hi; ++e) {
    const int iz = (int)(e % h);
    const size_t r = e / h;
    const int iy = (int)(r % n), ix = (int)(r / n);
    const long mx = ix <= n / 2 ? ix : ix - n, my = iy <= n / 2 ? iy : iy - n, mz = iz;
    const long m2 = mx * mx + my * my + mz * mz;
    if (m2 == 0) continue;
    int bin = (int)sqrt((double)m2);  // floor(sqrt(m2)), corrected to the exact integer
    while ((long)(bin + 1) * (bin + 1) <= m2) ++bin;
    while ((long)bin * bin > m2) --bin;
    if (bin >= nbins) continue;
    if (bin != cur) {
      flush();
      cur = bin;
    }
    const double w = (iz == 0 || 2 * iz == n) ? 1.0 : 2.0;
    const float2 av = a[e], bv = b[e];
    acc[0] += w;
    acc[1] += w * ((double)av.x * av.x + (double)av.y * av.y);
    acc[2] += w * ((double)bv.x * bv.x + (double)bv.y * bv.y);
    acc[3] += w * ((double)av.x * bv.x + (double)av.y * bv.y);
  }
  flush();
}

// out[q][bin] = sum over threads of work[q][bin][t] (fixed tree); spectra normalised by the
// mode count and L^3 / n^6 once the count is known (q = 0 block of each bin does it).
__global__ __launch_bounds__(TB) void power_reduce_kernel(const double* __restrict__ work,
                                                          int nbins, double norm,
                                                          double* __restrict__ out) {
  __shared__ double sh[TB];
  const int bin = blockIdx.x;
  double s[4];
  for (int q = 0; q < 4; ++q) {
    double acc = 0.0;
    const double* src = work + ((size_t)q * nbins + bin) * PS_THREADS;
    for (int t = threadIdx.x; t < PS_THREADS; t += TB) acc += src[t];
    s[q] = block_sum(acc, sh);
  }
  if (threadIdx.x == 0) {
    const double c = s[0];
    out[bin] = c;
    for (int q = 1; q < 4; ++q) out[(size_t)q * nbins + bin] = c > 0 ? s[q] * norm / c : 0.0;
  }
}

}  // namespace

size_t vec_work_doubles(size_t n) { return (size_t)dot_blocks(n) + 64; }

void launch_vec_dot(size_t n, const float* a, const float* b, const double* den, double* out,
                    double* work, hipStream_t s) {
  const int nb = dot_blocks(n);
  dot_partial_kernel<<<nb, TB, 0, s>>>(a, b, n, work);
  dot_final_kernel<<<1, TB, 0, s>>>(work, nb, den, out);
}

void launch_vec_axpby(size_t n, float alpha, const float* a, float beta, const float* b,
                      float* out, hipStream_t s) {
  axpby_kernel<<<stream_grid(n), TB, 0, s>>>(n, alpha, a, beta, b, out);
}

// d = -H g by the two-loop recursion. order[0..count): history slots, newest first. sy, yy:
// s.y and y.y per slot (device). scal: 2 m + 2 device doubles (alpha per slot, beta).
void launch_lbfgs_direction(size_t n, int m, int count, const int* order, const float* S,
                            const float* Y, const double* sy, const double* yy, const float* g,
                            float* d, double* work, double* scal, hipStream_t s) {
  const unsigned gs = stream_grid(n);
  axpby_kernel<<<gs, TB, 0, s>>>(n, 1.f, g, 0.f, g, d);  // q = g
  double* alpha = scal;
  double* beta = scal + m;
  for (int j = 0; j < count; ++j) {  // newest to oldest
    const int i = order[j];
    launch_vec_dot(n, S + (size_t)i * n, d, sy + i, alpha + i, work, s);  // alpha_i = s.q / s.y
    axpy_dev_kernel<<<gs, TB, 0, s>>>(n, alpha + i, nullptr, -1.0, Y + (size_t)i * n, d);
  }
  if (count > 0) scale_dev_kernel<<<gs, TB, 0, s>>>(n, sy + order[0], yy + order[0], 1.0, d);
  for (int j = count - 1; j >= 0; --j) {  // oldest to newest
    const int i = order[j];
    launch_vec_dot(n, Y + (size_t)i * n, d, sy + i, beta, work, s);  // beta = y.r / s.y
    axpy_dev_kernel<<<gs, TB, 0, s>>>(n, alpha + i, beta, 1.0, S + (size_t)i * n, d);
  }
  axpby_kernel<<<gs, TB, 0, s>>>(n, -1.f, d, 0.f, d, d);
}

size_t power_work_doubles(int nbins) { return (size_t)4 * nbins * PS_THREADS; }

void launch_power_bins(int n, double box, const float2* a, const float2* b, int nbins,
                       double* out, double* work, hipStream_t s) {
  const size_t total = (size_t)n * n * (n / 2 + 1);
  const size_t chunk = (total + PS_THREADS - 1) / PS_THREADS;
  power_partial_kernel<<<PS_THREADS / TB, TB, 0, s>>>(n, a, b, nbins, chunk, work);
  const double norm = box * box * box / ((double)n * n * n * (double)n * n * n);
  power_reduce_kernel<<<nbins, TB, 0, s>>>(work, nbins, norm, out);
}

}  // namespace pmr

// ---------------------------------------------------------------- fixed scratch
// The scratch of pmr_lbfgs_direction_noalloc: the partial sums of one inner product
// (vec_work_doubles(n) <= DOT_BLOCKS + 64) followed by the two-loop scalars (alpha per slot,
// beta: at most 2 * 64 + 8). One copy per GPU, held until the process ends; every call on a
// GPU shares it, so calls that overlap on one GPU (several streams or threads) race.
constexpr int NOALLOC_MAX_M = 64;
constexpr size_t NOALLOC_DOUBLES = (size_t)pmr::DOT_BLOCKS + 64 + 2 * NOALLOC_MAX_M + 8;
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};  // device address of `scratch` on each GPU

// Device address of this GPU's copy of `scratch` (the GPU that runs `stream`), taken once per
// device with that device current. In host code the array's name is only a stand-in for
// the symbol, so kernels get this address instead.
int scratch_of(hipStream_t stream, double** out) {
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess) return PMR_E_HIP;
  int dev = cur;
  if (stream && hipStreamGetDevice(stream, &dev) != hipSuccess) return PMR_E_HIP;
  if (dev < 0 || dev >= kMaxDevices) return PMR_E_SHAPE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    if (dev != cur && hipSetDevice(dev) != hipSuccess) return PMR_E_HIP;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (dev != cur) (void)hipSetDevice(cur);
    if (e != hipSuccess || !p) return PMR_E_HIP;
    g_scratch_dev[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_dev[dev];
  return PMR_OK;
}
}  // namespace

// ---------------------------------------------------------------- C ABI
using namespace pmr;

extern "C" {

size_t pmr_vec_work_bytes(size_t n, int m) {
  if (m < 0) return 0;
  return (vec_work_doubles(n) + (size_t)m + 8) * sizeof(double);
}

int pmr_vec_dot(size_t n, const float* a, const float* b, double* out, void* work, void* stream) {
  if (!a || !b || !out || !work || n == 0) return PMR_E_INVALID;
  launch_vec_dot(n, a, b, nullptr, out, (double*)work, (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? PMR_OK : PMR_E_HIP;
}

int pmr_vec_axpby(size_t n, double alpha, const float* a, double beta, const float* b,
                  float* out, void* stream) {
  if (!a || !b || !out || n == 0) return PMR_E_INVALID;
  launch_vec_axpby(n, (float)alpha, a, (float)beta, b, out, (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? PMR_OK : PMR_E_HIP;
}

int pmr_lbfgs_direction(size_t n, int m, int count, const int* order, const float* S,
                        const float* Y, const double* sy, const double* yy, const float* g,
                        float* d, void* work, void* stream) {
  if (!g || !d || !work || n == 0 || g == d || m < 1 || m > 64 || count < 0 || count > m)
    return PMR_E_INVALID;
  if (count > 0) {
    if (!order || !S || !Y || !sy || !yy) return PMR_E_INVALID;
    unsigned long long seen = 0;
    for (int j = 0; j < count; ++j) {
      if (order[j] < 0 || order[j] >= m || (seen >> order[j]) & 1ull) return PMR_E_INVALID;
      seen |= 1ull << order[j];
    }
  }
  double* w = (double*)work;
  launch_lbfgs_direction(n, m, count, order, S, Y, sy, yy, g, d, w, w + vec_work_doubles(n),
                         (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? PMR_OK : PMR_E_HIP;
}

int pmr_lbfgs_direction_noalloc(size_t n, int m, int count, const int* order, const float* S,
                                const float* Y, const double* sy, const double* yy,
                                const float* g, float* d, void* stream) {
  if (!g || !d || n == 0 || g == d || m < 1 || count < 0 || count > m) return PMR_E_INVALID;
  if (m > NOALLOC_MAX_M) return PMR_E_SHAPE;  // the fixed scratch holds 2 m + 2 scalars
  if (count > 0) {
    if (!order || !S || !Y || !sy || !yy) return PMR_E_INVALID;
    unsigned long long seen = 0;
    for (int j = 0; j < count; ++j) {
      if (order[j] < 0 || order[j] >= m || (seen >> order[j]) & 1ull) return PMR_E_INVALID;
      seen |= 1ull << order[j];
    }
  }
  hipStream_t s = (hipStream_t)stream;
  double* w = nullptr;
  const int st = scratch_of(s, &w);
  if (st != PMR_OK) return st;
  const size_t part = vec_work_doubles(n);
  if (part + 2 * (size_t)m + 2 > NOALLOC_DOUBLES) return PMR_E_SHAPE;
  launch_lbfgs_direction(n, m, count, order, S, Y, sy, yy, g, d, w, w + part, s);
  return hipGetLastError() == hipSuccess ? PMR_OK : PMR_E_HIP;
}

size_t pmr_power_work_bytes(int nbins) {
  if (nbins < 1) return 0;
  return power_work_doubles(nbins) * sizeof(double);
}

int pmr_power_bins(int n, double box, const void* a, const void* b, int nbins, double* out,
                   void* work, size_t work_bytes, void* stream) {
  if (!a || !b || !out || !work || !(box > 0)) return PMR_E_INVALID;
  if (n < 2 || n > 1024 || (n & (n - 1)) != 0 || nbins < 1 || nbins > 2 * n) return PMR_E_SHAPE;
  if (work_bytes < pmr_power_work_bytes(nbins)) return PMR_E_WORKSPACE;
  launch_power_bins(n, box, (const float2*)a, (const float2*)b, nbins, out, (double*)work,
                    (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? PMR_OK : PMR_E_HIP;
}

}  // extern "C"
