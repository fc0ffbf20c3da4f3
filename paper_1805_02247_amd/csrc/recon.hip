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

// The loop bodies below are shared by the kernels with host scalars and the kernels of the
// device-driven optimiser, so both evaluate every element with the same operations: a
// rounded FP32 product then one fused multiply-add, products exact in FP64.

// partial[block] = sum over this block's grid-stride elements of a[i] b[i] (FP64).
__device__ __forceinline__ void dot_partial_body(const float* __restrict__ a,
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
__device__ __forceinline__ void dot_final_body(const double* __restrict__ partial, int np,
                                               const double* __restrict__ den,
                                               double* __restrict__ out) {
  __shared__ double sh[TB];
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += TB) acc += partial[i];
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) out[0] = den ? s / den[0] : s;
}

__device__ __forceinline__ void axpy_body(size_t n, float c, const float* __restrict__ x,
                                          float* __restrict__ y) {
  const size_t stride = (size_t)gridDim.x * TB;
  for (size_t i = (size_t)blockIdx.x * TB + threadIdx.x; i < n; i += stride)
    y[i] = __fmaf_rn(c, x[i], y[i]);
}

__device__ __forceinline__ void scale_body(size_t n, float c, float* __restrict__ x) {
  const size_t stride = (size_t)gridDim.x * TB;
  for (size_t i = (size_t)blockIdx.x * TB + threadIdx.x; i < n; i += stride) x[i] *= c;
}

__device__ __forceinline__ void axpby_body(size_t n, float alpha, const float* a, float beta,
                                           const float* b, float* out) {
  const size_t stride = (size_t)gridDim.x * TB;
  for (size_t i = (size_t)blockIdx.x * TB + threadIdx.x; i < n; i += stride)
    out[i] = __fmaf_rn(beta, b[i], __fmul_rn(alpha, a[i]));
}

__global__ __launch_bounds__(TB) void dot_partial_kernel(const float* __restrict__ a,
                                                         const float* __restrict__ b, size_t n,
                                                         double* __restrict__ partial) {
  dot_partial_body(a, b, n, partial);
}

__global__ __launch_bounds__(TB) void dot_final_kernel(const double* __restrict__ partial, int np,
                                                       const double* __restrict__ den,
                                                       double* __restrict__ out) {
  dot_final_body(partial, np, den, out);
}

// y += sign * (A - B) * x with A, B device scalars (B nullable).
__global__ __launch_bounds__(TB) void axpy_dev_kernel(size_t n, const double* __restrict__ A,
                                                      const double* __restrict__ B, double sign,
                                                      const float* __restrict__ x,
                                                      float* __restrict__ y) {
  axpy_body(n, (float)(sign * (A[0] - (B ? B[0] : 0.0))), x, y);
}

// x *= sign * num / den (device scalars).
__global__ __launch_bounds__(TB) void scale_dev_kernel(size_t n, const double* __restrict__ num,
                                                       const double* __restrict__ den, double sign,
                                                       float* __restrict__ x) {
  scale_body(n, (float)(sign * num[0] / den[0]), x);
}

// out = alpha a + beta b (host scalars; out may alias a or b).
__global__ __launch_bounds__(TB) void axpby_kernel(size_t n, float alpha, const float* a,
                                                   float beta, const float* b, float* out) {
  axpby_body(n, alpha, a, beta, b, out);
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

// ---------------------------------------------------------------- device-driven L-BFGS
// Every kernel below reads the optimiser state first and returns at once (all threads
// alike) unless the state is in the phase it belongs to; so a fixed sequence of launches --
// capturable as a graph -- performs whichever branch the device-side tests chose.
namespace {

enum Gate {
  G_RUN = 0,   // the stage is running
  G_ACC = 1,   // the last trial was accepted (the pair and the move to x_t)
  G_DIR = 2,   // accepted and still running (the next direction)
  G_RESET = 3  // ... and that direction was not a descent direction
};
constexpr int NO_SLOT = -1;   // the vector as given
constexpr int NEW_SLOT = -2;  // slot of the candidate pair (state.slot)
// j >= 0: history entry j, slot state.order[j]; a kernel with jc >= 0 runs only while
// jc < state.count.

__device__ __forceinline__ bool gate_open(const pmr_lbfgs_state* st, int gate, int jc) {
  bool on;
  if (gate == G_RUN)
    on = st->status == PMR_LBFGS_RUNNING;
  else if (gate == G_ACC)
    on = st->accepted != 0;
  else if (gate == G_DIR)
    on = st->accepted != 0 && st->status == PMR_LBFGS_RUNNING;
  else
    on = st->accepted != 0 && st->status == PMR_LBFGS_RUNNING && st->reset != 0;
  return on && (jc < 0 || jc < st->count);
}

__device__ __forceinline__ size_t slot_of(const pmr_lbfgs_state* st, int j) {
  return j == NO_SLOT ? 0 : (size_t)(j == NEW_SLOT ? st->slot : st->order[j]);
}

__device__ __forceinline__ double* f_hist(pmr_lbfgs_state* st) {
  return reinterpret_cast<double*>(st + 1);
}
__device__ __forceinline__ long long* clock_hist(pmr_lbfgs_state* st) {
  return reinterpret_cast<long long*>(f_hist(st) + st->p.max_iter + 1);
}

__global__ __launch_bounds__(TB) void lb_dot_partial_kernel(const pmr_lbfgs_state* st, int gate,
                                                            int jc, const float* A, int ja,
                                                            const float* B, int jb, size_t n,
                                                            double* partial) {
  if (!gate_open(st, gate, jc)) return;
  dot_partial_body(A + slot_of(st, ja) * n, B + slot_of(st, jb) * n, n, partial);
}

__global__ __launch_bounds__(TB) void lb_dot_final_kernel(const pmr_lbfgs_state* st, int gate,
                                                          int jc, const double* partial, int np,
                                                          const double* den, int jden,
                                                          double* out, int jout) {
  if (!gate_open(st, gate, jc)) return;
  dot_final_body(partial, np, den ? den + slot_of(st, jden) : nullptr, out + slot_of(st, jout));
}

// y += sign * (A[slot] - B) * X[slot]
__global__ __launch_bounds__(TB) void lb_axpy_kernel(const pmr_lbfgs_state* st, int gate, int jc,
                                                     size_t n, const double* A, int ja,
                                                     const double* B, double sign,
                                                     const float* X, int jx, float* y) {
  if (!gate_open(st, gate, jc)) return;
  axpy_body(n, (float)(sign * (A[slot_of(st, ja)] - (B ? B[0] : 0.0))), X + slot_of(st, jx) * n,
            y);
}

// x *= sign * num[slot] / den[slot]
__global__ __launch_bounds__(TB) void lb_scale_kernel(const pmr_lbfgs_state* st, int gate, int jc,
                                                      size_t n, const double* num,
                                                      const double* den, int j, double sign,
                                                      float* x) {
  if (!gate_open(st, gate, jc)) return;
  const size_t i = slot_of(st, j);
  scale_body(n, (float)(sign * num[i] / den[i]), x);
}

// out[slot] = alpha a + beta b
__global__ __launch_bounds__(TB) void lb_axpby_kernel(const pmr_lbfgs_state* st, int gate, int jc,
                                                      size_t n, float alpha, const float* a,
                                                      float beta, const float* b, float* out,
                                                      int jout) {
  if (!gate_open(st, gate, jc)) return;
  axpby_body(n, alpha, a, beta, b, out + slot_of(st, jout) * n);
}

// xt = x + t d
__global__ __launch_bounds__(TB) void lb_trial_kernel(const pmr_lbfgs_state* st, size_t n,
                                                      const float* x, const float* d, float* xt) {
  if (st->status != PMR_LBFGS_RUNNING) return;
  axpby_body(n, 1.f, x, (float)st->t, d, xt);
}

__global__ void lb_init_kernel(pmr_lbfgs_state* st, pmr_lbfgs_params p, const double* loss,
                               long long clock_khz) {
  st->p = p;
  st->clock_khz = clock_khz;
  st->f = loss[0];
  st->ft = st->f;
  st->t = 0.0;
  st->gd = st->gg = st->rel = st->ss = st->beta = 0.0;
  st->status = PMR_LBFGS_RUNNING;
  st->iters = 0;
  st->evals = 1;
  st->count = 0;
  st->halvings = 0;
  st->probe = 1;
  st->accepted = 1;  // opens the direction kernels that follow
  st->slot = 0;
  st->reset = 0;
  f_hist(st)[0] = st->f;
  clock_hist(st)[0] = wall_clock64();
}

// a zero gradient ends the stage
__global__ void lb_gg_kernel(pmr_lbfgs_state* st) {
  if (!gate_open(st, G_DIR, -1)) return;
  if (st->gg == 0.0) st->status = PMR_LBFGS_STATIONARY;
}

// not a descent direction: clear the history, d = -g follows
__global__ void lb_gd_kernel(pmr_lbfgs_state* st) {
  if (!gate_open(st, G_DIR, -1)) return;
  if (st->gd >= 0.0) {
    st->count = 0;
    st->reset = 1;
    st->gd = -st->gg;
  } else {
    st->reset = 0;
  }
}

// first trial step of the search
__global__ void lb_step_kernel(pmr_lbfgs_state* st) {
  if (!gate_open(st, G_DIR, -1)) return;
  st->probe = st->count == 0;
  st->t = st->probe ? __ddiv_rn(1.0, __dsqrt_rn(st->gg)) : 1.0;
  st->halvings = 0;
}

// Armijo test of the trial; on rejection halve t, on acceptance pick the candidate slot
__global__ void lb_test_kernel(pmr_lbfgs_state* st, const double* loss) {
  if (st->status != PMR_LBFGS_RUNNING) {
    st->accepted = 0;
    return;
  }
  st->evals += 1;
  st->ft = loss[0];
  const double bound = __dadd_rn(st->f, __dmul_rn(__dmul_rn(st->p.c1, st->t), st->gd));
  st->accepted = st->ft <= bound;
  if (!st->accepted) {
    st->t *= 0.5;
    if (++st->halvings > st->p.max_halvings) st->status = PMR_LBFGS_LINE_SEARCH;
    return;
  }
  for (int k = 0; k <= st->p.m; ++k) {
    bool used = false;
    for (int j = 0; j < st->count; ++j) used = used || st->order[j] == k;
    if (!used) {
      st->slot = k;
      break;
    }
  }
}

// curvature test, history update, the move to x_t and the stopping rules
__global__ void lb_accept_kernel(pmr_lbfgs_state* st, const double* sy, const double* yy) {
  if (!gate_open(st, G_ACC, -1)) return;
  const int i = st->slot;
  if (sy[i] > __dmul_rn(st->p.curvature_eps, __dsqrt_rn(__dmul_rn(yy[i], st->ss)))) {
    const int keep = st->count < st->p.m ? st->count : st->p.m - 1;
    for (int k = keep; k > 0; --k) st->order[k] = st->order[k - 1];
    st->order[0] = i;
    st->count = keep + 1;
  }
  st->rel = st->f != 0.0 ? __ddiv_rn(__dsub_rn(st->f, st->ft), fabs(st->f)) : 0.0;
  st->f = st->ft;
  st->iters += 1;
  f_hist(st)[st->iters] = st->f;
  clock_hist(st)[st->iters] = wall_clock64();
  if (st->f <= st->p.stop_below)
    st->status = PMR_LBFGS_TARGET;
  else if (st->rel < st->p.rel_tol && !st->probe)
    st->status = PMR_LBFGS_CONVERGED;
  else if (st->iters >= st->p.max_iter)
    st->status = PMR_LBFGS_MAX_ITER;
}

}  // namespace

// FP64 inner product out[jout] = A[ja] . B[jb] (/ den[jden]) under a gate.
void lb_dot(const pmr_lbfgs_state* st, int gate, int jc, size_t n, const float* A, int ja,
            const float* B, int jb, const double* den, int jden, double* out, int jout,
            double* work, hipStream_t s) {
  const int nb = dot_blocks(n);
  lb_dot_partial_kernel<<<nb, TB, 0, s>>>(st, gate, jc, A, ja, B, jb, n, work);
  lb_dot_final_kernel<<<1, TB, 0, s>>>(st, gate, jc, work, nb, den, jden, out, jout);
}

// The next direction at x (g): the zero-gradient test, the two-loop recursion over the
// device-held history, the descent test with its fallback d = -g, and the first step.
void lb_direction(pmr_lbfgs_state* st, size_t n, int m, const float* g, float* d, const float* S,
                  const float* Y, const double* sy, const double* yy, double* work,
                  hipStream_t s) {
  const unsigned gs = stream_grid(n);
  lb_dot(st, G_DIR, -1, n, g, NO_SLOT, g, NO_SLOT, nullptr, NO_SLOT, &st->gg, NO_SLOT, work, s);
  lb_gg_kernel<<<1, 1, 0, s>>>(st);
  lb_axpby_kernel<<<gs, TB, 0, s>>>(st, G_DIR, -1, n, 1.f, g, 0.f, g, d, NO_SLOT);  // q = g
  for (int j = 0; j < m; ++j) {  // newest to oldest: alpha_i = s_i.q / s_i.y_i; q -= alpha_i y_i
    lb_dot(st, G_DIR, j, n, S, j, d, NO_SLOT, sy, j, st->alpha, j, work, s);
    lb_axpy_kernel<<<gs, TB, 0, s>>>(st, G_DIR, j, n, st->alpha, j, nullptr, -1.0, Y, j, d);
  }
  lb_scale_kernel<<<gs, TB, 0, s>>>(st, G_DIR, 0, n, sy, yy, 0, 1.0, d);  // r = gamma q
  for (int j = m - 1; j >= 0; --j) {  // oldest to newest: beta = y_i.r / s_i.y_i
    lb_dot(st, G_DIR, j, n, Y, j, d, NO_SLOT, sy, j, &st->beta, NO_SLOT, work, s);
    lb_axpy_kernel<<<gs, TB, 0, s>>>(st, G_DIR, j, n, st->alpha, j, &st->beta, 1.0, S, j, d);
  }
  lb_axpby_kernel<<<gs, TB, 0, s>>>(st, G_DIR, -1, n, -1.f, d, 0.f, d, d, NO_SLOT);
  lb_dot(st, G_DIR, -1, n, g, NO_SLOT, d, NO_SLOT, nullptr, NO_SLOT, &st->gd, NO_SLOT, work, s);
  lb_gd_kernel<<<1, 1, 0, s>>>(st);
  lb_axpby_kernel<<<gs, TB, 0, s>>>(st, G_RESET, -1, n, -1.f, g, 0.f, g, d, NO_SLOT);
  lb_step_kernel<<<1, 1, 0, s>>>(st);
}

void launch_lbfgs_init(size_t n, const pmr_lbfgs_params& p, pmr_lbfgs_state* st,
                       const double* loss, const float* g, float* d, const float* S,
                       const float* Y, const double* sy, const double* yy, double* work,
                       long long clock_khz, hipStream_t s) {
  lb_init_kernel<<<1, 1, 0, s>>>(st, p, loss, clock_khz);
  lb_direction(st, n, p.m, g, d, S, Y, sy, yy, work, s);
}

void launch_lbfgs_trial(size_t n, const pmr_lbfgs_state* st, const float* x, const float* d,
                        float* xt, hipStream_t s) {
  lb_trial_kernel<<<stream_grid(n), TB, 0, s>>>(st, n, x, d, xt);
}

void launch_lbfgs_update(size_t n, int m, pmr_lbfgs_state* st, const double* loss, float* x,
                         float* g, const float* xt, const float* gt, float* d, float* S,
                         float* Y, double* sy, double* yy, double* work, hipStream_t s) {
  const unsigned gs = stream_grid(n);
  lb_test_kernel<<<1, 1, 0, s>>>(st, loss);
  lb_axpby_kernel<<<gs, TB, 0, s>>>(st, G_ACC, -1, n, 1.f, xt, -1.f, x, S, NEW_SLOT);
  lb_axpby_kernel<<<gs, TB, 0, s>>>(st, G_ACC, -1, n, 1.f, gt, -1.f, g, Y, NEW_SLOT);
  lb_dot(st, G_ACC, -1, n, S, NEW_SLOT, Y, NEW_SLOT, nullptr, NO_SLOT, sy, NEW_SLOT, work, s);
  lb_dot(st, G_ACC, -1, n, Y, NEW_SLOT, Y, NEW_SLOT, nullptr, NO_SLOT, yy, NEW_SLOT, work, s);
  lb_dot(st, G_ACC, -1, n, S, NEW_SLOT, S, NEW_SLOT, nullptr, NO_SLOT, &st->ss, NO_SLOT, work, s);
  lb_accept_kernel<<<1, 1, 0, s>>>(st, sy, yy);
  lb_axpby_kernel<<<gs, TB, 0, s>>>(st, G_ACC, -1, n, 1.f, xt, 0.f, xt, x, NO_SLOT);
  lb_axpby_kernel<<<gs, TB, 0, s>>>(st, G_ACC, -1, n, 1.f, gt, 0.f, gt, g, NO_SLOT);
  lb_direction(st, n, m, g, d, S, Y, sy, yy, work, s);
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

size_t pmr_lbfgs_state_bytes(int max_iter) {
  if (max_iter < 1) return 0;
  return sizeof(pmr_lbfgs_state) + (size_t)(max_iter + 1) * (sizeof(double) + sizeof(long long));
}

int pmr_lbfgs_init(size_t n, const pmr_lbfgs_params* params, void* state, const double* loss,
                   const float* g, float* d, const float* S, const float* Y, const double* sy,
                   const double* yy, void* work, void* stream) {
  if (!params || !state || !loss || !g || !d || !S || !Y || !sy || !yy || !work || n == 0 ||
      g == d)
    return PMR_E_INVALID;
  const pmr_lbfgs_params& p = *params;
  if (p.m < 1 || p.m > PMR_LBFGS_MAX_M || p.max_iter < 1 || p.max_halvings < 0 ||
      !(p.c1 > 0.0 && p.c1 < 1.0) || !(p.curvature_eps >= 0.0) || !(p.rel_tol >= 0.0) ||
      p.stop_below != p.stop_below)
    return PMR_E_INVALID;
  hipStream_t s = (hipStream_t)stream;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PMR_E_HIP;
  if (s && hipStreamGetDevice(s, &dev) != hipSuccess) return PMR_E_HIP;
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
    return PMR_E_HIP;
  launch_lbfgs_init(n, p, (pmr_lbfgs_state*)state, loss, g, d, S, Y, sy, yy, (double*)work, khz,
                    s);
  return hipGetLastError() == hipSuccess ? PMR_OK : PMR_E_HIP;
}

int pmr_lbfgs_trial(size_t n, const void* state, const float* x, const float* d, float* xt,
                    void* stream) {
  if (!state || !x || !d || !xt || n == 0 || xt == x || xt == d) return PMR_E_INVALID;
  launch_lbfgs_trial(n, (const pmr_lbfgs_state*)state, x, d, xt, (hipStream_t)stream);
  return hipGetLastError() == hipSuccess ? PMR_OK : PMR_E_HIP;
}

int pmr_lbfgs_update(size_t n, int m, void* state, const double* loss, float* x, float* g,
                     const float* xt, const float* gt, float* d, float* S, float* Y, double* sy,
                     double* yy, void* work, void* stream) {
  if (!state || !loss || !x || !g || !xt || !gt || !d || !S || !Y || !sy || !yy || !work ||
      n == 0 || m < 1 || m > PMR_LBFGS_MAX_M || g == d || xt == x || gt == g)
    return PMR_E_INVALID;
  launch_lbfgs_update(n, m, (pmr_lbfgs_state*)state, loss, x, g, xt, gt, d, S, Y, sy, yy,
                      (double*)work, (hipStream_t)stream);
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
