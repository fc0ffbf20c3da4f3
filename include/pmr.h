/*
 * pmr.h - differentiable particle-mesh forward model and its adjoint on one MI355X (gfx950).
 *
 * The problem is the one of Sec. 5 (Reconstruction) of Modi, Feng & Seljak (2018): a forward
 * model f(s) maps the linear density modes s to a halo-mass field; the loss of Sec. 5.1,
 * Eq. (loss), adds the Gaussian prior of Eq. (priorpdf) to the displaced log-normal
 * likelihood of Eqs. (var) and (probnoise); the optimiser of Sec. 5.2 needs dL/ds for every
 * mode. The forward model is a Zel'dovich start, an n-step particle-mesh evolution (Sec. 3),
 * the features of Sec. 2.2 and the per-voxel network of Sec. 2.1.
 *
 * Conventions
 *   - Modes and gradients: interleaved complex float32 in real-FFT storage
 *     [B][Np][Np][Np/2+1] (C order, unnormalised forward DFT: s(k) = sum_x d(x) e^{-i k.x}).
 *     Every stored real and imaginary part is a parameter: grad = dL/dRe(s) + i dL/dIm(s).
 *     Input modes are projected onto the half spectrum of a real field (the kz = 0 and
 *     kz = Np/2 planes are averaged with the conjugate of their (-kx, -ky) partner, k = 0
 *     is removed) before use.
 *   - Meshes: float32 [B][N][N][N] C order, node i at position i * box / N.
 *   - Particles start on a lattice offset by half a force-mesh cell from the mesh nodes.
 *
 * Ownership: every array argument is a DEVICE pointer owned by the caller, including the
 * workspace passed to pmr_create. The library never allocates device memory. set_* calls
 * copy their inputs into the workspace (stream-ordered), so the caller may reuse its
 * buffers once the stream has passed the call. All calls enqueue work on the context's
 * stream and return without synchronising it, except where a declaration says otherwise
 * (pmr_set_check_finite, pmr_profile_end). Small host arrays (loss parameters, noise
 * tables) are passed to the device as kernel arguments, so they need not outlive the call.
 *
 * Errors: calls return PMR_OK or a negative status and never abort. Argument and shape
 * errors are detected synchronously. A HIP launch or runtime error is reported as
 * PMR_E_HIP and is sticky for the context.
 *
 * Threading: a context belongs to one stream; calls on one context are not re-entrant.
 */
#ifndef PMR_H
#define PMR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  PMR_OK = 0,
  PMR_E_INVALID = -1,   /* null pointer or invalid value */
  PMR_E_SHAPE = -2,     /* unsupported sizes */
  PMR_E_WORKSPACE = -3, /* workspace too small or misaligned (256 B) */
  PMR_E_HIP = -4,       /* HIP runtime or launch error (sticky) */
  PMR_E_NONFINITE = -5, /* non-finite loss (only with pmr_set_check_finite on; not sticky) */
  PMR_E_STATE = -6      /* call out of order (adjoint before forward, missing inputs) */
};

enum { PMR_FP32 = 0, PMR_MIXED = 1 };
enum { PMR_LOSS_DENSITY_L2 = 0, PMR_LOSS_LOGNORMAL = 1 };
/* Halo model of the log-normal loss: one softplus network on the voxel's features, or the
 * paper's product of a position network and a mass network (Sec. 2, Sec. 2.1). */
enum { PMR_HALO_SINGLE = 0, PMR_HALO_TWO = 1 };
/* Floats of the packed weight blocks of the two networks (pmr_set_halo_nets). */
enum { PMR_NNP_FLOATS = 50 * 81 + 50 + 30 * 50 + 30 + 30 + 1, PMR_NNM_FLOATS = 20 * 3 + 20 + 10 * 20 + 10 + 10 + 1 };

typedef struct pmr_config {
  int batch;      /* independent realisations B >= 1 */
  int n_part;     /* particles per axis Np: power of two, 16..512 */
  int n_mesh;     /* force mesh per axis: Np or 2 Np, <= 512 */
  int n_out;      /* output (halo-model) mesh per axis: Np or n_mesh */
  int n_steps;    /* kick-drift-kick steps, uniform in a, >= 1 */
  int mlp_hidden; /* hidden width H of the 3 -> H -> H -> 1 network: 8, 16, 32 or 64
                     (PMR_HALO_SINGLE; ignored by PMR_HALO_TWO) */
  int precision;  /* PMR_FP32, or PMR_MIXED (network on BF16 matrix cores) */
  int ckpt_every; /* 0: keep every step for the adjoint; k >= 1: keep (x, p) every k steps
                     and recompute the steps in between during the adjoint */
  int loss_kind;  /* PMR_LOSS_LOGNORMAL (Sec. 5.1) or PMR_LOSS_DENSITY_L2 */
  double box;     /* periodic box side, Mpc/h */
  double a0, a1;  /* start and end scale factors (0 < a0 < a1) */
  double omega_m; /* flat LambdaCDM matter density (Sec. 3: 0.3175) */
  double R1, R2;  /* Gaussian feature scales, Mpc/h (Sec. 2.2) */
  int ic_order;   /* initial conditions (Sec. 3): 0 or 1 first-order (Zel'dovich) displacement,
                     2 second-order LPT (adds 3/7 D0^2 Psi2 to x0 and 6/7 D0 Gp0 Psi2 to p0) */
  int halo_model; /* PMR_HALO_SINGLE, or PMR_HALO_TWO (log-normal loss and PMR_FP32 only) */
} pmr_config;

/* Loss parameters of one batch item (Sec. 5.1, Eq. loss; Sec. 5.2 anneals R_sm and M0). */
typedef struct pmr_loss_params {
  double M0;           /* nuisance mass added before the log, Eq. (var) */
  double mu;           /* offset mu_N of the displaced log-normal */
  double sigma_N;      /* width sigma_N (residual = (mu + x - x_data) / (2 sigma_N)) */
  double R_mass;       /* Gaussian smoothing of model and data mass fields, Mpc/h */
  double R_sm;         /* residual smoothing of the anneal, Mpc/h (0 = none) */
  double prior_weight; /* weight of the prior term (1 for Eq. loss) */
  double logistic_a;   /* sharpness a of the position network's logistic, Eq. logistic
                          (PMR_HALO_TWO; Sec. 5.2 anneals it 1 -> 2 -> 3); > 0 */
} pmr_loss_params;

typedef struct pmr_ctx pmr_ctx;

/* Bytes of device workspace needed for `cfg`; 0 if the configuration is invalid. */
size_t pmr_workspace_bytes(const pmr_config* cfg);

/* Create a context on `stream` (a hipStream_t; NULL = default stream) over a caller-owned
 * device workspace of at least pmr_workspace_bytes(cfg) bytes, 256-byte aligned. The
 * kick/drift factors and growth functions are computed on the host here (FP64). */
int pmr_create(const pmr_config* cfg, void* workspace, size_t workspace_bytes, void* stream,
               pmr_ctx** out);
int pmr_set_stream(pmr_ctx* ctx, void* stream);
int pmr_destroy(pmr_ctx* ctx);

/* Prior inverse variance 1/S(k) per stored mode, float32 [Np][Np][Np/2+1], shared by all
 * items; S = <|s(k)|^2> (Eq. priorpdf); use 0 at k = 0. Copied. */
int pmr_set_prior(pmr_ctx* ctx, const float* inv_var);

/* Network weights, float32 row-major [out][in]: W1 [H][3], b1 [H], W2 [H][H], b2 [H],
 * W3 [1][H], b3 [1] (Sec. 2.1; frozen). Copied. Required for PMR_LOSS_LOGNORMAL. */
int pmr_set_mlp(pmr_ctx* ctx, const float* W1, const float* b1, const float* W2,
                const float* b2, const float* W3, const float* b3);

/* Weights of the two-network halo model (Sec. 2: model = NNp x NNm; Sec. 2.1), device
 * float32, each network packed as its layers in order, weights row-major [out][in]:
 *   nnp (PMR_NNP_FLOATS): W1 [50][81], b1 [50], W2 [30][50], b2 [30], W3 [1][30], b3 [1];
 *     ReLU hidden layers, output logistic(y, a) with a the loss parameter logistic_a;
 *     input feature c * 27 + o is feature field c (delta_0, delta_R1, delta_R1 - delta_R2)
 *     at the voxel displaced by (dx, dy, dz) = (o / 9 - 1, (o / 3) % 3 - 1, o % 3 - 1),
 *     periodic (Sec. 2.2: the 3 x 3 x 3 neighbourhood);
 *   nnm (PMR_NNM_FLOATS): W1 [20][3], b1 [20], W2 [10][20], b2 [10], W3 [1][10], b3 [1];
 *     ELU hidden layers (Eq. elu), linear output, on the voxel's own three features.
 * The modelled mass NNp x NNm must keep M_R + M0 > 0 for the log of the likelihood.
 * Copied (stream-ordered). PMR_E_STATE unless the context was created with PMR_HALO_TWO. */
int pmr_set_halo_nets(pmr_ctx* ctx, const float* nnp, const float* nnm);

/* Data field [B][Nout^3]: the halo mass field (log-normal loss) or the target density
 * contrast (density-L2 loss). Copied. */
int pmr_set_target(pmr_ctx* ctx, const float* target);

/* Loss parameters (Sec. 5.1, Eq. loss; the anneal stages of Sec. 5.2 change R_sm, M0 and
 * the logistic sharpness a), HOST array [B]. Checked here (PMR_E_INVALID: sigma_N <= 0,
 * M0 <= 0 for the log-normal loss, negative R, non-finite mu or prior_weight, a <= 0 with
 * PMR_HALO_TWO) and stored in device memory stream-ordered, without synchronising; the data
 * term x_data = log(G_Rmass * M_target + M0) is recomputed on the stream. Kernels read the
 * parameters from device memory, so a forward captured in a HIP graph picks up a later
 * pmr_set_loss at its next replay. */
int pmr_set_loss(pmr_ctx* ctx, const pmr_loss_params* params);

/* The same from DEVICE memory: params_device is a [B] array of pmr_loss_params (8-byte
 * aligned) that the stream reads when it reaches this call, so the call itself can be
 * captured in a HIP graph and the caller may write new values into the array between
 * replays (the anneal stages of Sec. 5.2 without host synchronisation). The values are
 * checked on the device with the rules of pmr_set_loss; an item that fails them gets a NaN
 * loss (total, prior and data) from the next pmr_forward instead of an error status.
 * PMR_E_INVALID for a null or misaligned pointer. */
int pmr_set_loss_device(pmr_ctx* ctx, const pmr_loss_params* params_device);

/* Mass-dependent noise of the log-normal likelihood (Sec. 5.1: mu_N and sigma_N of Eq.
 * (probnoise) depend on the smoothed data mass M_R at the cell). HOST arrays of n_nodes
 * (<= 64): nodes log_mass (natural log of M_R of the data, strictly increasing) and the
 * values mu and sigma (> 0) there. Each cell takes the linear interpolation at
 * log(M_R,data), constant beyond the end nodes, for every batch item; this replaces the
 * scalar mu and sigma_N of pmr_set_loss. n_nodes = 0 restores the scalars. Copied to the
 * device as kernel arguments (stream-ordered, no synchronisation).
 * Whether a table is in use is fixed into a forward pass captured in a HIP graph: capture
 * after switching it on or off (changing the values of a table in use needs no recapture). */
int pmr_set_noise_table(pmr_ctx* ctx, int n_nodes, const double* log_mass, const double* mu,
                        const double* sigma);

/* Forward model and loss. modes: complex64 [B][Np][Np][Np/2+1] (device).
 * mass_out: [B][Nout^3] model mass field (log-normal) or final density contrast
 * (density-L2); nullable. loss_out: device double [B][3] = (total, prior, data).
 * Keeps what the adjoint needs in the workspace; invalidated by the next forward. */
int pmr_forward(pmr_ctx* ctx, const void* modes, float* mass_out, double* loss_out);

/* Number of pmr_forward calls enqueued on this context so far (or PMR_E_INVALID for a null
 * context). A caller that keeps the value of a forward can tell whether a later forward has
 * replaced the state its adjoint would use. */
long long pmr_forward_count(const pmr_ctx* ctx);

/* Optional check of the loss: with on != 0, pmr_forward synchronises the context stream at
 * its end, reads the B x 3 loss values back and returns PMR_E_NONFINITE if any is NaN or
 * infinite (its outputs are still written and pmr_adjoint may follow). Off by default; keep
 * it off while a forward is being captured into a HIP graph (the check synchronises). */
int pmr_set_check_finite(pmr_ctx* ctx, int on);

/* Gradient of sum_b loss_bar[b] * loss[b] + <mass_bar, mass> with respect to the modes of
 * the preceding pmr_forward. loss_bar: device double [B]; mass_bar: device float
 * [B][Nout^3] or NULL; grad_modes: complex64, same layout as the modes. Without
 * checkpointing (ckpt_every = 0, or ckpt_every >= n_steps) the adjoint may be called again
 * for the same forward; when it had to recompute checkpoint segments, the per-step state of
 * the last segment is gone and a further call returns PMR_E_STATE until the next
 * pmr_forward. */
int pmr_adjoint(pmr_ctx* ctx, const double* loss_bar, const float* mass_bar, void* grad_modes);

const char* pmr_status_string(int status);

/* ---- inspection of the last forward/adjoint (tests and profiling) ----
 * Copies an internal buffer of item-major layout into `dst` (device). Returns the number
 * of bytes copied, or a negative status. `step` selects the PM step where relevant.
 *   PMR_DBG_X         positions x_step, double [B][3][Np^3] (step 0..n; only the steps the
 *                     checkpoint policy keeps: all for ckpt_every = 0)
 *   PMR_DBG_FORCE     force mesh at x_step, interleaved float [B][Nm^3][3] = (Fx, Fy, Fz)
 *                     (same availability)
 *   PMR_DBG_SORT_IDS  sorted particle ids for x_step on the force mesh, u32 [B*Np^3]
 *   PMR_DBG_DELTA_F   final density contrast on the output mesh, float [B][Nout^3]
 *   PMR_DBG_FEATURES  (delta_R1, delta_R2), float [2][B][Nout^3]
 *   PMR_DBG_MASS_R    smoothed model mass M_R, float [B][Nout^3]
 *   PMR_DBG_RES_S     smoothed residual, float [B][Nout^3]
 *   PMR_DBG_XBAR0     adjoint of x0 after pmr_adjoint, float [B][3][Np^3]
 *   PMR_DBG_PBAR0     adjoint of p0 after pmr_adjoint, float [B][3][Np^3]
 *   PMR_DBG_DBAR_F    adjoint of the final density contrast, float [B][Nout^3]
 */
enum {
  PMR_DBG_X = 1,
  PMR_DBG_FORCE = 2,
  PMR_DBG_SORT_IDS = 3,
  PMR_DBG_DELTA_F = 4,
  PMR_DBG_FEATURES = 5,
  PMR_DBG_MASS_R = 6,
  PMR_DBG_RES_S = 7,
  PMR_DBG_XBAR0 = 8,
  PMR_DBG_PBAR0 = 9,
  PMR_DBG_DBAR_F = 10
};
long long pmr_debug_copy(pmr_ctx* ctx, int what, int step, void* dst);

/* ---- event timing of one kernel class (measurement) ----
 * Between pmr_profile_begin and pmr_profile_end, every launch of `kernel_class` enqueued by
 * pmr_forward / pmr_adjoint on this context is bracketed by a pair of HIP events on the
 * context stream (at most `max_launches` launches are recorded; events are created on the
 * host at the first call). pmr_profile_end synchronises the stream and returns the summed
 * event time, the number of launches and their summed algorithmic bytes (the compulsory
 * HBM traffic of each launch: inputs read once, outputs written once). */
enum {
  PMR_PROF_NONE = 0,
  PMR_PROF_PAINT = 1,             /* density paint on the force mesh (one channel) */
  PMR_PROF_XPASS_FORCE = 2,       /* outermost-axis pass with the force operator: the x
                                     component and the potential, 1 -> 2 */
  PMR_PROF_YPASS = 3,             /* middle-axis FFT passes, with the y and z derivatives of
                                     the potential (force) and their transposes (adjoint) */
  PMR_PROF_ZPASS = 4,             /* contiguous-axis r2c / c2r passes */
  PMR_PROF_KICK_DRIFT = 5,        /* readout + kick + drift + keys */
  PMR_PROF_PAINT3 = 6,            /* three-channel adjoint paint */
  PMR_PROF_XPASS_FORCE_ADJ = 7,   /* outermost-axis pass with the force adjoint: the x
                                     channel and the y pass's combination of y and z, 2 -> 1 */
  PMR_PROF_ADJ_GATHER = 8,        /* step-adjoint position gradient (sorted-order gather) */
  PMR_PROF_ADJ_UPDATE = 9,        /* step-adjoint kick / drift transposes (id order) */
  PMR_PROF_HALO2 = 10,            /* two-network model kernels (forward, adjoint); their
                                     algorithmic figure is FLOPs, not bytes */
  PMR_PROF_HALO2_STENCIL = 11,    /* two-network model: neighbourhood sum of the position
                                     network's input adjoint */
  PMR_PROF_SORT = 13,             /* every kernel of one cell-key sort and its row index, as
                                     one launch; an implementation cost that serves the paint
                                     and the adjoint gathers: its algorithmic bytes are 0 */
  PMR_PROF_NETWORK = 14           /* the single network's forward and adjoint kernels; their
                                     algorithmic figure is FLOPs: 2 (4H + H^2) per voxel
                                     forward, 2 (8H + 2H^2) adjoint (recomputed activations
                                     and the transposed products) */
};
int pmr_profile_begin(pmr_ctx* ctx, int kernel_class, int max_launches);
int pmr_profile_end(pmr_ctx* ctx, double* total_ms, long long* launches, double* alg_bytes);

/* ---- stand-alone hot-path primitives (device pointers, enqueued on `stream`) ---- */

/* Unnormalised forward 3-D real FFT of `batch` fields [batch][n^3] -> [batch][n][n][n/2+1]
 * (the numpy rfftn convention). n: power of two 16..512. */
int pmr_fft_r2c(int n, int batch, const float* in, void* out, void* stream);

/* Inverse 3-D real FFT including the 1/n^3 factor (numpy irfftn). The spectrum `inout`
 * is used as scratch and overwritten. Imaginary parts that a real field cannot carry
 * (kz = 0, n/2 columns after the inner transforms) are ignored, as irfftn does. */
int pmr_fft_c2r(int n, int batch, void* inout, float* out, void* stream);

/* Tile shape of one strided FFT pass for size n (process-wide; the autotuner sets it).
 * `pass` PMR_FFT_YPASS (the middle axis), PMR_FFT_XPASS (the outermost axis with a
 * single-input k-space operator: forward or inverse only, force, smoothing, Zel'dovich; also
 * the middle-axis pass that takes the y and z derivatives of the force's potential) or
 * PMR_FFT_XPASS_MULTI (the outermost axis with a multi-input operator: force adjoint, feature
 * adjoint, gradient assembly; also the middle-axis pass that combines the adjoint's y and z
 * channels). `columns` consecutive kz columns per workgroup tile
 * (8, 16 or 32) and `threads` per workgroup (256 or 512), with
 * threads <= n * columns <= 16 * threads and the tile within 160 KB of LDS. `staging` 0 runs
 * the butterflies on register images of the tile (radix-8 stages; used where n * columns /
 * threads is a multiple of 8 and n >= 64; LDS only permutes between radix stages), 1 runs
 * every stage on the LDS-staged tile with radix-8 stages (then one radix-4 or radix-2
 * stage), 2 the same with radix-4 stages (then one radix-2 stage). Invalid values return
 * PMR_E_INVALID and leave the shape unchanged.
 * Defaults: 16 columns, 256 threads, staging 0. Not synchronised with work in flight: set it
 * before enqueueing. */
enum { PMR_FFT_YPASS = 0, PMR_FFT_XPASS = 1, PMR_FFT_XPASS_MULTI = 2 };
int pmr_fft_set_tile(int n, int pass, int columns, int threads, int staging);
int pmr_fft_get_tile(int n, int pass, int* columns, int* threads, int* staging);

/* Slab width of the force transforms of the PM steps on an n^3 mesh (process-wide; the
 * autotuner sets it): with `columns` > 0 the middle-axis pass, the outermost-axis pass with
 * its k-space operator and the inverse middle-axis passes run window by window of that many
 * kz columns (rounded up to a multiple of every strided pass's tile columns), so that a
 * window's spectra stay in the memory-side cache between the passes; 0 runs each pass
 * over the whole half spectrum. The results are the same bit for bit. `columns`: 0 or a
 * power of two up to 512; PMR_E_INVALID otherwise. Default 0. Not synchronised with work in
 * flight: set it before enqueueing. */
int pmr_fft_set_slab(int n, int columns);
int pmr_fft_get_slab(int n, int* columns);

/* Rows per wavefront of the CIC paints on an n^3 mesh with `channels` channels (1: the
 * density, 3: the adjoint's three force channels), process-wide; the autotuner sets it.
 * A wavefront owns `rows` consecutive target rows of one plane and walks the source rows
 * that reach them: more rows read each particle fewer times (2 (rows + 1) / rows walks)
 * but leave fewer wavefronts to share the dense rows of late steps. rows: 0 (the default
 * rule: 1024 floats of rows per wavefront, at most 8 rows), 1, 2, 4, 8 or 16; a value the
 * size cannot take (LDS, rows per plane) falls back to the default. Each value gives
 * bitwise reproducible results; different values group a cell's deposits differently and
 * differ by FP32 rounding. PMR_E_INVALID for other values. Not synchronised with work in
 * flight: set it before enqueueing. */
int pmr_paint_set_rows(int n, int channels, int rows);
int pmr_paint_get_rows(int n, int channels, int* rows);

/* Bytes of scratch for pmr_cic_sort with `n_particles` in total and `batch` items. */
size_t pmr_sort_scratch_bytes(int n_particles_total, int n_mesh, int batch);

/* Cell keys and the stable (key, id) order of positions x: double [B][3][Np^3].
 * key = item * n_mesh^3 + (ix * n_mesh + iy) * n_mesh + iz with i = floor(x * n_mesh / box)
 * mod n_mesh (FP64). Outputs (u32): keys_sorted [B*Np^3], ids_sorted [B*Np^3] (global ids
 * item * Np^3 + id) and row_start [B * n_mesh^2 + 1] (first sorted index of each row). */
int pmr_cic_sort(int n_part, int n_mesh, int batch, double box, const double* x,
                 uint32_t* keys_sorted, uint32_t* ids_sorted, uint32_t* row_start,
                 void* scratch, size_t scratch_bytes, void* stream);

/* CIC density on an n_mesh^3 mesh: out = sum_p mass W(x_p - cell) - bias, [B][n_mesh^3],
 * from the outputs of pmr_cic_sort. Deterministic (bitwise reproducible). `scratch` holds
 * the sorted fraction stream: at least 12 * B * Np^3 bytes. */
int pmr_cic_paint(int n_part, int n_mesh, int batch, double box, const double* x,
                  const uint32_t* keys_sorted, const uint32_t* ids_sorted,
                  const uint32_t* row_start, float mass, float bias, float* out, void* scratch,
                  size_t scratch_bytes, void* stream);

/* ---- reconstruction driver support ----
 * The optimiser of Sec. 5.2 is L-BFGS over all stored real and imaginary parts of the
 * modes; its inner products run in FP64 on the device and its scalars stay in device
 * memory, so a direction costs no host synchronisation. Vectors are float arrays of n
 * elements (a complex64 mode array is 2 x n_modes floats). Reductions use a fixed grid and
 * a fixed tree: bitwise reproducible. All calls enqueue on `stream` (a hipStream_t or NULL)
 * and return without synchronising; errors are PMR_E_INVALID for bad arguments. */

/* Bytes of device scratch `work` for pmr_vec_dot and pmr_lbfgs_direction on n floats with
 * a history of m pairs (m = 0 for pmr_vec_dot). */
size_t pmr_vec_work_bytes(size_t n, int m);

/* out[0] (device double) = sum_i a[i] b[i], products and sums in FP64. */
int pmr_vec_dot(size_t n, const float* a, const float* b, double* out, void* work, void* stream);

/* out = alpha a + beta b elementwise (FP32; host scalars; out may alias a or b). */
int pmr_vec_axpby(size_t n, double alpha, const float* a, double beta, const float* b,
                  float* out, void* stream);

/* L-BFGS search direction d = -H g (two-loop recursion; Nocedal & Wright, Numerical
 * Optimization, Alg. 7.4) with H0 = gamma I, gamma = s.y / y.y of the newest pair.
 * S, Y: device [m][n] floats, the history pairs s = x_{k+1} - x_k, y = g_{k+1} - g_k in
 * slots 0..m-1; order: HOST int array of `count` distinct slots, newest first; sy, yy:
 * device doubles [m] with s.y and y.y of each slot (pmr_vec_dot). count = 0 gives d = -g.
 * g and d must not alias. */
int pmr_lbfgs_direction(size_t n, int m, int count, const int* order, const float* S,
                        const float* Y, const double* sy, const double* yy, const float* g,
                        float* d, void* work, void* stream);

/* pmr_lbfgs_direction without the `work` argument, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight optimiser loops, harnesses that forbid it):
 * the FP64 partial sums and the two-loop scalars live in a fixed array inside the library,
 * one per GPU (1224 doubles, about 10 KB: up to 1088 partial sums and 2 m + 2 scalars),
 * held until the process ends; the call allocates nothing and frees nothing. Same arguments, rules and results
 * (bit for bit) as pmr_lbfgs_direction; PMR_E_SHAPE for m > 64 (beyond the fixed array),
 * PMR_E_HIP if the array's address on the stream's GPU cannot be taken. All calls on one
 * GPU share the array: calls that overlap on one GPU (several streams or host threads)
 * race and must be serialised by the caller. */
int pmr_lbfgs_direction_noalloc(size_t n, int m, int count, const int* order, const float* S,
                                const float* Y, const double* sy, const double* yy,
                                const float* g, float* d, void* stream);

/* ---- L-BFGS with its line search on the device (Sec. 5.2) ----
 * One optimiser iteration as device work only, so that a whole evaluation -- trial point,
 * forward, adjoint, Armijo test, history update, next direction -- can be one HIP-graph
 * replay with no host round trip; the host reads the status block every few replays.
 * The rules are those of the host driver: the first step of a stage (or after a
 * non-descent direction clears the history) has length one along -g (t = 1 / |g|), later
 * searches start at t = 1; a trial at step t is accepted when f(x + t d) <= f + c1 t g.d,
 * else t is halved, and the search fails after max_halvings + 1 rejected trials; an
 * accepted step (s = x_t - x, y = g_t - g) enters the history (newest first, at most m
 * pairs; the oldest leaves) only if s.y > curvature_eps |s| |y|; the stage ends when the
 * relative decrease (f - f_t) / |f| of an accepted step falls below rel_tol (not for the
 * unit probe step), when f_t <= stop_below, at a zero gradient, or after max_iter accepted
 * steps. Scalars are FP64 in device memory, with the products, sums, square roots and
 * quotients of those tests rounded once each in the order written above, so the decisions
 * and iterates equal, bit for bit, those of a host driver evaluating the same expressions
 * in FP64 on the same losses and inner products.
 *
 * state: device buffer of pmr_lbfgs_state_bytes(max_iter) bytes. It starts with a
 * pmr_lbfgs_state (the host may copy that prefix back to read status, iters, evals, f)
 * followed by f_hist[max_iter + 1] (double: the loss after each accepted step, f_hist[0]
 * at the start) and clock_hist[max_iter + 1] (long long: the device wall clock, at
 * clock_khz ticks per ms, when each was reached). A zeroed state is PMR_LBFGS_IDLE, in
 * which pmr_lbfgs_trial and pmr_lbfgs_update do nothing. S, Y: device [m + 1][n] floats
 * (the history and one slot for the candidate pair); sy, yy: device doubles [m + 1]; work:
 * pmr_vec_work_bytes(n, 0) bytes. All calls enqueue kernels only (no copies, no memsets)
 * and return without synchronising. */
enum {
  PMR_LBFGS_IDLE = 0,        /* zeroed state: trial and update do nothing */
  PMR_LBFGS_RUNNING = 1,
  PMR_LBFGS_CONVERGED = 2,   /* relative decrease below rel_tol */
  PMR_LBFGS_STATIONARY = 3,  /* g = 0 */
  PMR_LBFGS_LINE_SEARCH = 4, /* max_halvings + 1 rejected trials */
  PMR_LBFGS_MAX_ITER = 5,
  PMR_LBFGS_TARGET = 6       /* loss at or below stop_below */
};
enum { PMR_LBFGS_MAX_M = 64 };

typedef struct pmr_lbfgs_params {
  int m;              /* history pairs, 1..PMR_LBFGS_MAX_M */
  int max_iter;       /* accepted steps per stage, >= 1 */
  int max_halvings;   /* >= 0 */
  double c1;          /* Armijo constant */
  double curvature_eps;
  double rel_tol;
  double stop_below;  /* -INFINITY for none */
} pmr_lbfgs_params;

typedef struct pmr_lbfgs_state {
  double f;       /* loss at the current point x */
  double t;       /* step of the next trial */
  double gd;      /* g.d at x */
  double gg;      /* g.g at x */
  double rel;     /* relative decrease of the last accepted step */
  double ft;      /* loss at the last trial */
  double ss;      /* s.s of the last candidate pair */
  double beta;    /* two-loop scratch */
  int status;     /* PMR_LBFGS_* */
  int iters;      /* accepted steps */
  int evals;      /* evaluations: the starting one and every trial */
  int count;      /* history pairs held */
  int halvings;   /* rejected trials of the current search */
  int probe;      /* the current search is the unit-length probe step */
  int accepted;   /* the last trial was accepted */
  int slot;       /* slot of the last candidate pair */
  int reset;      /* the last direction was not a descent direction */
  int pad;
  long long clock_khz;
  pmr_lbfgs_params p;
  int order[PMR_LBFGS_MAX_M];          /* history slots, newest first */
  double alpha[PMR_LBFGS_MAX_M + 1];   /* two-loop scalars per slot */
} pmr_lbfgs_state;

size_t pmr_lbfgs_state_bytes(int max_iter);

/* Starts a stage at x from the loss (device double) and gradient g at x: history cleared,
 * f_hist[0] = loss, then the first direction (d = -g) and t = 1 / |g| (PMR_LBFGS_STATIONARY
 * at g = 0). PMR_E_INVALID for bad parameters or pointers, PMR_E_HIP if the device clock
 * rate cannot be read. */
int pmr_lbfgs_init(size_t n, const pmr_lbfgs_params* params, void* state, const double* loss,
                   const float* g, float* d, const float* S, const float* Y, const double* sy,
                   const double* yy, void* work, void* stream);

/* xt = x + t d with the state's t, while the state is PMR_LBFGS_RUNNING (else nothing). */
int pmr_lbfgs_trial(size_t n, const void* state, const float* x, const float* d, float* xt,
                    void* stream);

/* After the evaluation at xt (its loss, device double, and gradient gt): the Armijo test;
 * on acceptance the candidate pair, the curvature test and history update, x = xt,
 * g = gt, the stopping rules and the next direction in d with its t; on rejection t is
 * halved. m must equal the params' m given to pmr_lbfgs_init. Nothing while the state is
 * not PMR_LBFGS_RUNNING. */
int pmr_lbfgs_update(size_t n, int m, void* state, const double* loss, float* x, float* g,
                     const float* xt, const float* gt, float* d, float* S, float* Y, double* sy,
                     double* yy, void* work, void* stream);

/* Bytes of device scratch for pmr_power_bins with `nbins` shells. */
size_t pmr_power_work_bytes(int nbins);

/* Binned auto and cross power of two half spectra a, b (complex64 [n][n][n/2+1], numpy
 * rfftn layout) of a box of side `box` (two point functions, Sec. 4.3). Shell i holds the
 * full-spectrum modes with i <= |m| < i + 1 (m the integer wavevector; k = 2 pi m / box),
 * the k = 0 mode excluded. out: device doubles [4][nbins] = (count, P_aa, P_bb, P_ab) with
 * P = box^3 / n^6 * mean over the shell's full-spectrum modes of |a|^2, |b|^2, Re a conj b
 * (0 for an empty shell). n: power of two 2..1024; 1 <= nbins <= 2 n. */
int pmr_power_bins(int n, double box, const void* a, const void* b, int nbins, double* out,
                   void* work, size_t work_bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* PMR_H */
