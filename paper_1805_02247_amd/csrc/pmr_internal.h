// Internal device/host helpers shared by the HIP translation units of libpmr.
// gfx950 (CDNA4) only: 64-lane wavefronts, 160 KB LDS per CU.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#define PMR_WAVE 64

namespace pmr {

// ------------------------------------------------------------------ complex
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by +i (dir > 0) or -i (dir < 0)
template <int DIR>
__device__ __forceinline__ float2 cmul_i(float2 a) {
  return DIR > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// ------------------------------------------------------------------ k-space helpers
// integer wavenumber of storage index i on an axis of n points (full axes)
__device__ __forceinline__ int wavenumber(int i, int n) { return i <= n / 2 ? i : i - n; }

// ------------------------------------------------------------------ CIC helpers
// Lower-corner index and fraction of one coordinate, FP64 (bit-identical rule everywhere):
// u = x * scale, fl = floor(u), i0 = (int)fl mod n, f = u - fl, each operation rounded on
// its own. Contraction is off here: fused into f = fma(x, scale, -fl) in some kernels and
// not in others, the fraction of one position would differ in its last bits between the
// kernel that first computes it and the one that recomputes it from the stored position.
__device__ __forceinline__ int cic_corner(double x, double scale, int n, double* frac) {
#pragma clang fp contract(off)
  double u = x * scale;
  double fl = floor(u);
  *frac = u - fl;
  return (int)fl & (n - 1);  // floor(u) mod n (n a power of two; also for negative floor)
}

__device__ __forceinline__ double wrap_box(double x, double box) {
#pragma clang fp contract(off)
  return x - box * floor(x / box);
}

// Workgroups of a 1-D grid are dispatched round-robin over the 8 XCDs of the chip, each
// with its own L2. Remapping the block index gives every XCD one contiguous range of
// logical blocks, so spatially neighbouring work shares an L2. Bijective for any nb.
// Workgroups of `kernel` (launched with `threads` threads and no dynamic LDS) that the
// current device holds at once: occupancy per CU (registers, LDS, waves) times the CUs.
// Persistent tile loops launch this many, so that no workgroup waits for a second round.
// Computed once per kernel (and block size); the library runs on one device model per process.
inline int resident_grid_of(const void* kernel, int threads) {
  int per_cu = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus < 1)
    cus = 256;
  return per_cu * cus;
}

template <auto Kernel, int Threads>
inline int resident_grid() {
  static const int grid = resident_grid_of(reinterpret_cast<const void*>(Kernel), Threads);
  return grid;
}

__device__ __forceinline__ int xcd_block(int b, int nb) {
  constexpr int X = 8;
  const int q = nb / X, r = nb % X;
  const int x = b % X, i = b / X;
  return x * q + (x < r ? x : r) + i;
}

}  // namespace pmr

// ------------------------------------------------------------------ launch declarations
// (defined in the .hip files; all enqueue on `stream`, no synchronisation)
namespace pmr {

// Addressing of the fields of a batched pass: field f belongs to item f / fpi and is
// component f % fpi of it.
struct FieldMap {
  int fpi;
  size_t item_stride, comp_stride;  // elements (of the array's type)
  size_t pitch;                     // spectra: complex elements per (x, y) row, >= n/2 + 1
  __host__ __device__ size_t off(int f) const {
    return (size_t)(f / fpi) * item_stride + (size_t)(f % fpi) * comp_stride;
  }
};

// Inputs of the CIC paint kernels: the particle streams in (key, id) order and the row index.
// Rows per wave of the paints: TY = min(PMR_PAINT_LDS_FLOATS / (N C), PMR_PAINT_TY_MAX),
// rounded down to a power of two. Fewer rows per wave balance the clustered rows of late
// steps across more waves, at the cost of re-reading one source row per TY target rows.
#ifndef PMR_PAINT_TY_MAX
#define PMR_PAINT_TY_MAX 8
#endif
#ifndef PMR_PAINT_LDS_FLOATS
#define PMR_PAINT_LDS_FLOATS 1024
#endif

// Three floats, 12 bytes: a cell of the force mesh (F_x, F_y, F_z), so that a CIC corner is
// one three-dword load, and an element of the per-particle streams (CIC fractions, adjoint
// paint values, position gradients).
struct Vec3 {
  float x, y, z;
};

struct PaintArgs {
  const uint32_t* keys;     // sorted keys
  const Vec3* frac;       // sorted fractions
  const Vec3* val;        // sorted values (C = 3), or nullptr (C = 1, constant mass)
  const uint32_t* row_start;
  int nm, log_nm;
  float mass, bias;
  float* out;               // [B][C][nm^3]
};

// Kinds of fused k-space operation performed in the outermost-axis pass.
enum XOp : int {
  XOP_FWD = 0,        // forward transform only (completes an r2c); 1 in -> 1 out (spectrum)
  XOP_INV = 1,        // inverse only, scaled by 1/n^3; 1 in (spectrum) -> 1 out
  XOP_FORCE = 2,      // fwd, * i k_a / k^2 / n^3, inv; 1 in -> 3 out
  XOP_FORCE_ADJ = 3,  // 3 in: fwd each, sum conj(i k_a / k^2) / n^3, inv; -> 1 out
  XOP_GAUSS = 4,      // fwd, * exp(-k^2 R_b^2 / 2) / n^3, inv; 1 in -> 1 out (R per batch item)
  XOP_GAUSS2 = 5,     // fwd, * exp(-k^2 R1^2/2)/n^3 and exp(-k^2 R2^2/2)/n^3, inv; 1 -> 2
  XOP_FEAT_ADJ = 6,   // 2 in (A, B): fwd, (G1 A - G2 B)/n^3, inv; -> 1 out
  XOP_ZA = 7,         // 1 in (projected modes, already spectral): * i k_a / k^2 / n^3, inv; -> 3
  XOP_ZA_ADJ = 8,     // 3 in: fwd, gradient assembly with the prior term; -> caller's gradient
  XOP_HESS = 9,       // 1 in (projected modes): * k_a k_b / k^2 / n^3, inv; -> 3 (pair set at
                      // param_index: 0 -> xx, yy, zz; 1 -> xy, xz, yz)
  XOP_HESS_ADJ = 10,  // 3 in (same pair sets): fwd, sum k_a k_b / k^2 / n^3; caller's gradient +=
  // The force split over the axes: a factor that depends on k_y or k_z only commutes with
  // the transform along x, so the x pass carries the x component and one potential, and
  // the y pass takes both of the potential's other derivatives, instead of three spectra
  // going through the x pass and back.
  XOP_FORCE_X = 11,      // fwd, * i k_x / k^2 / n^3 and * 1 / k^2 / n^3, inv; 1 in -> 2 out
  XOP_FORCE_X_ADJ = 12,  // 2 in (A, B): fwd each, (conj(i k_x) A + B) / k^2 / n^3, inv; -> 1 out
  // Operators on y lines (tile = kz chunk of one x plane; k_y and k_z enter):
  XOP_YGRAD = 13,      // 1 in (spectral along y): i k_y A and i k_z A, inverse y; 1 -> 2
  XOP_YGRAD_ADJ = 14,  // 2 in (A, B): forward y each, conj(i k_y) A + conj(i k_z) B; -> 1
                       // out (spectral)
};

// Loss parameters per batch item in device memory (doubles):
// M0, mu, sigma_N, R_mass, R_sm, prior_weight, logistic_a (the fields of the public struct,
// PMR_LOSS_FIELDS of them), then a validity slot (1: the item's values passed the checks).
constexpr int PMR_LOSS_FIELDS = 7;
constexpr int PRM_VALID = 7;
constexpr int NPRM = 8;
// Items per launch of the kernel that stores host parameters from its arguments.
constexpr int PRM_CHUNK = 32;
struct ParamChunk {
  double v[PRM_CHUNK * NPRM];
  int b0, count;
};

struct XPassArgs {
  int n;            // points per axis
  int batch;
  int n_in, n_out;
  const float2* in[3];
  float2* out[3];
  size_t in_item_stride, out_item_stride;  // complex elements between batch items
  size_t in_pitch, out_pitch;              // complex elements per (x, y) row of in / out
  size_t aux_item_stride;                  // for proj_modes (standard layout, pitch n/2 + 1)
  double box;
  double R1, R2;       // feature scales (XOP_GAUSS2 / XOP_FEAT_ADJ)
  const double* params;  // device loss params [B][NPRM] (XOP_GAUSS reads R at param_index)
  int param_index;
  // gradient assembly (XOP_ZA_ADJ, XOP_HESS_ADJ)
  const float2* proj_modes;  // P s
  const float* inv_var;      // 1 / S(k), shared by all items
  const double* loss_bar;    // [B]
  int kz_lo, kz_hi;          // kz window of the pass (kz_hi = 0: the whole half spectrum)
};

// z pass r2c over `fields` fields; loaded value = a1*in (+ a2*in2) (* scale_dev[item])
void launch_zpass_r2c(int n, int fields, const float* in, FieldMap im, const float* in2, float a1,
                      float a2, const double* scale_dev, float2* out, FieldMap om, hipStream_t s);
// z pass c2r (unnormalised); optional out += add (add uses the output map)
void launch_zpass_c2r(int n, int fields, const float2* in, FieldMap im, float* out, FieldMap om,
                      const float* add, hipStream_t s);
// Inverse z pass of the three components of a vector field per item (im: 3 fields per item)
// into one interleaved Vec3 mesh [item][n^3] = (f0, f1, f2).
// CIC paint of `channels` (1: mass, bias subtracted; 3: adjoint values) fused with the z pass
// of the r2c: writes the z-transformed half spectra of the painted meshes (om: fields per
// item = channels); the y and x passes complete the transform.
void launch_paint_r2c(int n, int channels, const PaintArgs& a, int batch, float2* out, FieldMap om,
                      hipStream_t s);
void launch_zpass_c2r3(int n, int items, const float2* in, FieldMap im, Vec3* out,
                       size_t out_item_stride, hipStream_t s);
// A window [lo, hi) of kz columns of the half spectrum (hi = 0: all of them).
struct KzWin {
  int lo = 0, hi = 0;
};
void launch_ypass(int n, int fields, float2* data, FieldMap m, bool inverse, hipStream_t s,
                  KzWin win = KzWin{});
void launch_xpass(int op, const XPassArgs& a, hipStream_t s);
// Tile shape of the strided passes (columns per tile, threads per workgroup, and whether the
// butterflies run on register images (0) or on the LDS-staged tile (1)), per pass (0: y pass,
// 1: x pass with a single-input operator, 2: x pass with a multi-input operator) and log2(n);
// set by pmr_fft_set_tile (the autotuner) or left at the defaults. Defined in fft.hip.
struct TileShape {
  int pc, nth, staging;  // staging: 0 registers, 1 LDS radix-8, 2 LDS radix-4
};
extern TileShape g_fft_tile[3][10];

// Rows per wavefront of the paints per size and channel count (1 or 3; 0: the default rule
// from PMR_PAINT_LDS_FLOATS and PMR_PAINT_TY_MAX); set by pmr_paint_set_rows (the autotuner).
int set_paint_rows(int n, int channels, int rows);
int get_paint_rows(int n, int channels);
int set_fft_tile(int n, int pass, int pc, int nth, int staging);
void get_fft_tile(int n, int pass, int* pc, int* nth, int* staging);
// kz-slab width of the strided passes per size (0: off); fft_slab_columns gives the width
// in use (a multiple of every pass's tile columns, 0 when one slab would hold everything).
int set_fft_slab(int n, int columns);
int get_fft_slab(int n);
int fft_slab_columns(int n);

// sort.hip: the unique (key, id) order of the id-order cell keys, sorted keys and ids, the
// row index row_start [rows + 1] (rows = key >> shift), pay_out[pos] = pay_in[id] and
// inv[id] = pos when given. `order` (nullable) is the order in which the particles are
// visited (a permutation of the ids, e.g. the previous step's sorted ids; it changes only
// the speed). Scratch of cell_sort_scratch_bytes(n, rows) bytes.
size_t cell_sort_scratch_bytes(int n, size_t rows, int shift);
void launch_cell_sort(const uint32_t* keys, const uint32_t* order, int n, int shift,
                      size_t rows, uint32_t* keys_sorted, uint32_t* ids_sorted,
                      uint32_t* row_start, void* scratch, const Vec3* pay_in, Vec3* pay_out,
                      uint32_t* inv, hipStream_t s);
// cic.hip
void launch_keys(const double* x, int log_np3, int total, double scale, int nm, uint32_t* keys,
                 Vec3* frac, hipStream_t s);
void launch_stream_frac(const uint32_t* ids, const double* x, int total, int log_np3, int nm,
                        double box, Vec3* frac, hipStream_t s);
void launch_stream_gather(const uint32_t* ids, const Vec3* src, int total, Vec3* dst,
                          hipStream_t s);
void launch_paint_mass(const uint32_t* keys, const Vec3* frac, const uint32_t* row_start,
                       int batch, int nm, float mass, float bias, float* out, hipStream_t s);
// F: interleaved force mesh [B][nm^3] of Vec3 (Fx, Fy, Fz). p = p_in + kick F (p_in
// nullable: p itself); p_ck (nullable) receives a second copy of the new p.
void launch_kick_drift(const double* x, double* x_next, const float* p_in, float* p,
                       float* p_ck, const Vec3* F, uint32_t* keys, Vec3* frac, int batch,
                       int log_np3, int nm, double box, float kick, double drift, int key_nm,
                       hipStream_t s);
// Position gradient of a step adjoint (or of the final paint: fbar = F = nullptr), computed in
// sort order and written to g_out in id order:
//   g = sum_corners dW/dx * (Fbar . F(corner) + mass * dbar(corner)).
void launch_adjoint_positions(const uint32_t* keys, const Vec3* frac, const Vec3* fbar,
                              const uint32_t* ids, const Vec3* F, const float* dbar, int total,
                              int nm, double box, float mass, Vec3* g_out, hipStream_t s);
// Kick and drift transposes with that gradient: pbar += drift xbar; xbar += g (final mode:
// xbar = g, pbar = 0); optionally the next reverse step's paint values into vnext, in id
// order, or in that step's sort order when vperm (its inverse permutation) is given.
void launch_adjoint_update(float* xbar, float* pbar, const Vec3* gpos, int batch, int log_np3,
                           float kick, float drift, int final_mode, Vec3* vnext, float kick_next,
                           float drift_next, const uint32_t* vperm, hipStream_t s);
// Initial positions and momenta from the first-order displacement psi and, when psi2 is
// not null, the second-order one: x = wrap(q + D0 psi + c2x psi2), p = Gp0 psi + c2p psi2.
void launch_za_init(const float* psi, const float* psi2, int batch, int np, int log_np3,
                    double box, double half_cell, double D0, float Gp0, double c2x, float c2p,
                    double* x, float* p, float* p_ck, uint32_t* keys, Vec3* frac, int key_nm,
                    hipStream_t s);
// Two-network halo model (halo2.hip). Prepared weight block of HALO2_WEIGHT_FLOATS floats.
constexpr int HALO2_WEIGHT_FLOATS = 448 + (4 * 21 + 2 * 16 + 4 * 8 + 6 * 16) * 64;
void launch_halo2_prepare(const float* nnp, const float* nnm, float* w, hipStream_t s);
// aux: [2][B][n^3] (pos, then m) and sgn: [B][n^3][4] ReLU signs, written by the forward
// and read by the adjoint.
void launch_halo2_fwd(const float* d0, const float* d1, const float* d2, int log_n, size_t total,
                      const float* w, const double* prm, float* aux, uint32_t* sgn, float* mass,
                      hipStream_t s);
// Writes u, the position network's input adjoint [B n^3 / 16][81][16] (16-voxel groups),
// and the mass network's input adjoint into (g0, g12, g2); launch_halo2_stencil_adj then
// adds the neighbourhood sums of u.
void launch_halo2_bwd(const float* d0, const float* d1, const float* d2, int log_n, size_t total,
                      const float* w, const double* prm, const float* mbar, const float* aux,
                      const uint32_t* sgn, float* u, float* g0, float* g12, float* g2,
                      hipStream_t s);
void launch_halo2_stencil_adj(const float* u, int log_n, size_t total, float* g0, float* g12,
                              float* g2, hipStream_t s);
// FMAs per voxel of the two-network kernels (forward; adjoint from the stored signs)
constexpr double HALO2_FWD_FMA = 81 * 50 + 50 * 30 + 30 + 3 * 20 + 20 * 10 + 10;
constexpr double HALO2_BWD_FMA = 30 * 50 + 50 * 81 + 3 * 20 + 20 * 10 + 10 + 10 * 20 + 20 * 3;
// Second-order LPT pointwise kernels (phi: [B][6][np^3], pairs xx, yy, zz, xy, xz, yz).
void launch_lpt2_source(const float* phi, int batch, int log_np3, float* S, size_t s_item_stride,
                        hipStream_t s);
void launch_lpt2_phi_bar(const float* phi, const float* Sbar, size_t s_item_stride, int batch,
                         int log_np3, float* phibar, hipStream_t s);

// halo.hip
size_t mlp_weight_floats(int H);
int launch_mlp_fwd(int H, const float* d0, const float* d1, const float* d2, size_t n,
                   const float* w, float* mass, hipStream_t s);
int launch_mlp_prepare_bf16(int H, float* w, hipStream_t s);
int launch_mlp_fwd_mfma(int H, const float* d0, const float* d1, const float* d2, size_t n,
                        const float* w, float* mass, hipStream_t s);
int launch_mlp_bwd_mfma(int H, const float* d0, const float* d1, const float* d2, size_t n,
                        const float* w, const float* mbar, float* g0, float* g12, float* g2,
                        hipStream_t s);
int launch_mlp_bwd(int H, const float* d0, const float* d1, const float* d2, size_t n,
                   const float* w, const float* mbar, float* g0, float* g12, float* g2,
                   hipStream_t s);
void launch_target_x(const float* mtr, size_t per_item, int batch, const double* prm, float* xd,
                     hipStream_t s);
void launch_residual(const float* mr, const float* xd, size_t per_item, int batch,
                     const double* prm, const float* nmu, const float* nw, float* r,
                     hipStream_t s);
void launch_mrbar(const float* rbar, const float* mr, size_t per_item, int batch,
                  const double* prm, const float* nw, float* out, hipStream_t s);
// Per-cell noise offset and 1 / (2 sigma) from the interpolation table (k nodes).
constexpr int NOISE_MAX = 64;
struct NoiseTable {
  double v[3 * NOISE_MAX];
};
// Loss parameters: from a host array of [batch][NPRM] doubles (passed as kernel arguments:
// no staging, no wait), or from device memory as the public struct array (checked there).
void launch_params_store(const double* host, int batch, double* prm, hipStream_t s);
void launch_params_from_device(const double* src, int batch, int density_l2, int halo_two,
                               double* prm, hipStream_t s);
void launch_noise_table_store(const double* host, double* tab, hipStream_t s);
void launch_noise_fields(const float* mrd, size_t total, const double* tab, int k, float* nmu,
                         float* nw, hipStream_t s);
void launch_l2_adj(const float* d, const float* t, size_t per_item, int batch,
                   const double* loss_bar, const float* extra, float* out, hipStream_t s);
int reduce_blocks(size_t per_item);
void launch_sumsq(const float* a, const float* c, size_t per_item, int batch, double* partial,
                  double* out, hipStream_t s);
void launch_project_prior(const float2* modes, int n, int batch, const float* inv_var, float2* ps,
                          double* partial, double* prior_out, hipStream_t s);
void launch_finalize_loss(const double* prior, const double* data, const double* prm, int batch,
                          double* loss_out, hipStream_t s);

}  // namespace pmr
