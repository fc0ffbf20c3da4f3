// C ABI of libpmr: configuration, workspace plan, growth factors and the forward/adjoint
// schedules. All device work is enqueued on the context's stream; nothing here allocates
// device memory.
#include "../../include/pmr.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "pmr_internal.h"

using namespace pmr;

namespace {

// ---------------------------------------------------------------- growth (host, FP64)
// Flat LambdaCDM: E(a) = sqrt(Om a^-3 + 1 - Om); D = C E(a) int_0^a da' / (a' E)^3,
// D(1) = 1; G_p = a^3 E dD/da. The integral is taken over t = sqrt(a') (a' = t^2), which
// makes the integrand smooth at 0, with adaptive Simpson.
struct Cosmo {
  double om;
  double E(double a) const { return std::sqrt(om / (a * a * a) + 1.0 - om); }
  double dE(double a) const { return -1.5 * om / (a * a * a * a) / E(a); }
  double integrand_t(double t) const {
    if (t <= 0.0) return 0.0;
    const double a = t * t;
    const double ae = a * E(a);
    return 2.0 * t / (ae * ae * ae);
  }
  double simpson(double lo, double hi, double flo, double fmid, double fhi, double whole,
                 double tol, int depth) const {
    const double mid = 0.5 * (lo + hi);
    const double lm = 0.5 * (lo + mid), rm = 0.5 * (mid + hi);
    const double flm = integrand_t(lm), frm = integrand_t(rm);
    const double left = (mid - lo) / 6.0 * (flo + 4.0 * flm + fmid);
    const double right = (hi - mid) / 6.0 * (fmid + 4.0 * frm + fhi);
    const double diff = left + right - whole;
    if (depth <= 0 || std::fabs(diff) <= 15.0 * tol) return left + right + diff / 15.0;
    return simpson(lo, mid, flo, flm, fmid, left, 0.5 * tol, depth - 1) +
           simpson(mid, hi, fmid, frm, fhi, right, 0.5 * tol, depth - 1);
  }
  double I(double a) const {
    const double hi = std::sqrt(a);
    const double f0 = integrand_t(0.0), f1 = integrand_t(0.5 * hi), f2 = integrand_t(hi);
    const double whole = hi / 6.0 * (f0 + 4.0 * f1 + f2);
    return simpson(0.0, hi, f0, f1, f2, whole, 1e-15, 40);
  }
  double norm() const { return E(1.0) * I(1.0); }
  double D(double a) const { return E(a) * I(a) / norm(); }
  double Gp(double a) const {
    const double dD = (dE(a) * I(a) + 1.0 / (a * a * a * E(a) * E(a))) / norm();
    return a * a * a * E(a) * dD;
  }
};

#define HIPC(c, call)                                        \
  do {                                                       \
    hipError_t e_ = (call);                                  \
    if (e_ != hipSuccess && (c)->status == PMR_OK) (c)->status = PMR_E_HIP; \
  } while (0)

bool pow2_in(int n, int lo, int hi) { return n >= lo && n <= hi && (n & (n - 1)) == 0; }
int ilog2(size_t v) {
  int l = 0;
  while (((size_t)1 << l) < v) ++l;
  return l;
}
size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace

// Row pitch of the library's internal half spectra, in complex elements: n/2 + 1 rounded up
// to 16 (128 bytes), so that every row of a strided FFT tile starts on a cache line. Arrays
// crossing the API (modes, gradient, prior table) keep the standard pitch n/2 + 1.
size_t spec_pitch(int n) { return ((size_t)(n / 2 + 1) + 15) / 16 * 16; }

struct pmr_ctx {
  pmr_config cfg;
  hipStream_t stream;
  char* ws;
  size_t ws_bytes;
  int status;       // sticky error
  int have_prior, have_mlp, have_target, have_loss, xd_dirty, fwd_done;
  int check_finite;  // pmr_set_check_finite
  long long n_forward;  // pmr_forward calls enqueued (pmr_forward_count)
  // sizes
  int B, np, nm, no, n, H, k;
  size_t np3, nm3, no3, cp, cm, co;  // standard half-spectrum sizes n * n * (n/2 + 1)
  size_t sp, sm, so, cmax;           // internal spectra: n * n * row pitch (rows of 128 B)
  int log_np3, log_nm, log_no;
  // factors
  double D0, Gp0;
  std::vector<double> kick, drift;
  float mass_m, mass_o;
  // device buffers
  float* inv_var;
  float* mlp_w;
  float* halo2_w;  // prepared weights of the two-network model
  float* u2;       // its position network's input adjoint [B no3 / 16][81][16]
  float* h2aux;    // its position mask and mass-network output [2][B][no3]
  uint32_t* h2sgn; // its position network's ReLU signs [B][no3][4]
  float* target;
  double* params;
  float* xd;
  double* noise_tab;   // [3][NOISE_MAX]: nodes in log(M_R,data), mu_N, sigma_N
  int noise_k;         // nodes in the table; 0: the scalar mu, sigma_N of the loss parameters
  float* noise_mu;     // per-cell mu_N [B][no3] (when noise_k > 0)
  float* noise_w;      // per-cell 1 / (2 sigma_N) [B][no3]
  float2* ps;
  double* xs;   // position slots [S][B][3][np3]
  int n_xslots;
  double* ckx;  // checkpoints [nck][B][3][np3]
  float* ckp;
  int n_ck;
  float* p;     // [B][3][np3]
  Vec3* F;    // force slots [SF][B][nm3], interleaved (Fx, Fy, Fz)
  uint32_t* ids;   // sort slots [SF][B*np3]
  uint32_t* skeys; // sorted keys [SF][B*np3]
  Vec3* frac;    // sorted CIC fractions [SF][B*np3]
  uint32_t* rows;  // [SF][B*nm*nm + 1]
  uint32_t* inv;   // inverse sort permutations (sorted position of each id) [SF][B*np3]
  int n_fslots;
  uint32_t* keys;
  uint32_t* keys_sorted;
  void* sort_scratch;
  size_t sort_scratch_bytes;
  uint32_t* ids_o;
  Vec3* frac_o;
  Vec3* frac_id;  // CIC fractions of the current positions, id order [B*np3]
  Vec3* vid;      // adjoint paint values of the next reverse step, id order [B*np3]
  Vec3* vstream;  // the same in sorted order [B*np3]
  Vec3* gpos;     // position gradient of the current step adjoint, id order [B*np3]
  uint32_t* rows_o;
  float2* cA;    // [B][cmax]
  float2* cB;    // [B][3][cmax]
  float* psi;    // [B][3][np3]
  float* psi2;   // second-order displacement [B][3][np3]; component 0 also holds S, S_bar
  float* phi;    // second derivatives of the linear potential [B][6][np3] (xx yy zz xy xz yz)
  float* phibar; // their adjoints [B][6][np3]
  float* delta_f;  // [B][no3]
  float* dR;       // [2][B][no3]
  float* mass;
  float* MR;
  float* r;
  float* rs;
  float* xbar;
  float* pbar;
  float* dbar;   // [B][nm3]
  float* ob;     // [4][B][no3]
  double* partial;
  double* prior;
  double* data;
  // event timing of one kernel class (pmr_profile_begin/end)
  int prof_class;
  std::vector<hipEvent_t> prof_ev;
  size_t prof_used;
  double prof_bytes;
  bool prof_open;  // a scatter-probe event pair is open
};

namespace {

int validate(const pmr_config* c) {
  if (!c) return PMR_E_INVALID;
  if (c->batch < 1 || c->n_steps < 1 || c->ckpt_every < 0) return PMR_E_INVALID;
  if (!pow2_in(c->n_part, 16, 512) || !pow2_in(c->n_mesh, 16, 512) || !pow2_in(c->n_out, 16, 512))
    return PMR_E_SHAPE;
  if (c->n_mesh != c->n_part && c->n_mesh != 2 * c->n_part) return PMR_E_SHAPE;
  if (c->n_out != c->n_part && c->n_out != c->n_mesh) return PMR_E_SHAPE;
  if (c->loss_kind != PMR_LOSS_DENSITY_L2 && c->loss_kind != PMR_LOSS_LOGNORMAL) return PMR_E_INVALID;
  if (c->halo_model != PMR_HALO_SINGLE && c->halo_model != PMR_HALO_TWO) return PMR_E_INVALID;
  const bool single = c->loss_kind == PMR_LOSS_LOGNORMAL && c->halo_model == PMR_HALO_SINGLE;
  if (single && c->mlp_hidden != 8 && c->mlp_hidden != 16 && c->mlp_hidden != 32 &&
      c->mlp_hidden != 64)
    return PMR_E_SHAPE;
  if (c->precision != PMR_FP32 && c->precision != PMR_MIXED) return PMR_E_INVALID;
  if (c->precision == PMR_MIXED && single && c->mlp_hidden != 32 && c->mlp_hidden != 64)
    return PMR_E_SHAPE;  // the matrix-core network tiles K in steps of 32
  if (c->halo_model == PMR_HALO_TWO &&
      (c->loss_kind != PMR_LOSS_LOGNORMAL || c->precision != PMR_FP32))
    return PMR_E_SHAPE;  // the two networks exist for the log-normal loss, in FP32
  if (!(c->box > 0) || !(c->a0 > 0) || !(c->a1 > c->a0) || !(c->omega_m > 0) || !(c->omega_m <= 1))
    return PMR_E_INVALID;
  if (!(c->R1 >= 0) || !(c->R2 >= 0)) return PMR_E_INVALID;
  if (c->ic_order < 0 || c->ic_order > 2) return PMR_E_INVALID;
  const double np3 = (double)c->n_part * c->n_part * c->n_part;
  const double nm3 = (double)c->n_mesh * c->n_mesh * c->n_mesh;
  const double no3 = (double)c->n_out * c->n_out * c->n_out;
  if (c->batch * np3 >= 2147483648.0) return PMR_E_SHAPE;  // int particle index
  if (c->batch * nm3 > 4294967296.0 || c->batch * no3 > 4294967296.0) return PMR_E_SHAPE;
  return PMR_OK;
}

// Workspace plan: a bump allocator that either measures (base == nullptr) or assigns.
struct Plan {
  char* base;
  size_t off;
  template <typename T>
  T* take(size_t count) {
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += align256(count * sizeof(T));
    return p;
  }
};

// The reverse step's paint values go straight into the next step's sort order (through the
// inverse sort permutation) only while the particle arrays stay cache-resident: both the
// inverse permutation and those values are random writes, which at 2^24 particles cost more
// (measured) than the coherent id-order write plus a sorted gather.
constexpr size_t kDirectSortedValuesMax = (size_t)1 << 23;
bool direct_sorted_values(const pmr_ctx* c) { return (size_t)c->B * c->np3 <= kDirectSortedValuesMax; }

void plan(pmr_ctx* c, Plan& P) {
  const size_t B = c->B;
  c->inv_var = P.take<float>(c->cp);
  c->mlp_w = P.take<float>(mlp_weight_floats(c->H > 0 ? c->H : 8));
  const bool two = c->cfg.halo_model == PMR_HALO_TWO;
  c->halo2_w = P.take<float>(two ? HALO2_WEIGHT_FLOATS : 0);
  c->u2 = P.take<float>(two ? 81 * B * c->no3 : 0);
  c->h2aux = P.take<float>(two ? 2 * B * c->no3 : 0);
  c->h2sgn = P.take<uint32_t>(two ? 4 * B * c->no3 : 0);
  c->target = P.take<float>(B * c->no3);
  c->params = P.take<double>(B * NPRM);
  c->xd = P.take<float>(B * c->no3);
  c->noise_tab = P.take<double>(3 * NOISE_MAX);
  c->noise_mu = P.take<float>(B * c->no3);
  c->noise_w = P.take<float>(B * c->no3);
  c->ps = P.take<float2>(B * c->cp);
  c->xs = P.take<double>((size_t)c->n_xslots * B * 3 * c->np3);
  c->ckx = P.take<double>((size_t)c->n_ck * B * 3 * c->np3);
  c->ckp = P.take<float>((size_t)c->n_ck * B * 3 * c->np3);
  c->p = P.take<float>(B * 3 * c->np3);
  c->F = P.take<Vec3>((size_t)c->n_fslots * B * c->nm3);
  c->ids = P.take<uint32_t>((size_t)c->n_fslots * B * c->np3);
  c->skeys = P.take<uint32_t>((size_t)c->n_fslots * B * c->np3);
  c->frac = P.take<Vec3>((size_t)c->n_fslots * B * c->np3);
  c->rows = P.take<uint32_t>((size_t)c->n_fslots * (B * c->nm * c->nm + 1));
  c->inv = P.take<uint32_t>(direct_sorted_values(c) ? (size_t)c->n_fslots * B * c->np3 : 0);
  c->keys = P.take<uint32_t>(B * c->np3);
  c->keys_sorted = P.take<uint32_t>(B * c->np3);
  {
    const size_t sm = cell_sort_scratch_bytes((int)(B * c->np3), B * c->nm * c->nm, c->log_nm);
    const size_t so = cell_sort_scratch_bytes((int)(B * c->np3), B * c->no * c->no, c->log_no);
    c->sort_scratch_bytes = sm > so ? sm : so;
  }
  c->sort_scratch = P.take<char>(c->sort_scratch_bytes);
  c->ids_o = P.take<uint32_t>(B * c->np3);
  c->frac_o = P.take<Vec3>(B * c->np3);
  c->frac_id = P.take<Vec3>(B * c->np3);
  c->vid = P.take<Vec3>(B * c->np3);
  c->vstream = P.take<Vec3>(B * c->np3);
  c->gpos = P.take<Vec3>(B * c->np3);
  c->rows_o = P.take<uint32_t>(B * c->no * c->no + 1);
  c->cA = P.take<float2>(B * c->cmax);
  c->cB = P.take<float2>(B * 3 * c->cmax);
  c->psi = P.take<float>(B * 3 * c->np3);
  const size_t l2 = c->cfg.ic_order == 2 ? B * c->np3 : 0;
  c->psi2 = P.take<float>(3 * l2);
  c->phi = P.take<float>(6 * l2);
  c->phibar = P.take<float>(6 * l2);
  c->delta_f = P.take<float>(B * c->no3);
  c->dR = P.take<float>(2 * B * c->no3);
  c->mass = P.take<float>(B * c->no3);
  c->MR = P.take<float>(B * c->no3);
  c->r = P.take<float>(B * c->no3);
  c->rs = P.take<float>(B * c->no3);
  c->xbar = P.take<float>(B * 3 * c->np3);
  c->pbar = P.take<float>(B * 3 * c->np3);
  c->dbar = P.take<float>(B * c->nm3);
  c->ob = P.take<float>(4 * B * c->no3);
  const size_t nred = (size_t)reduce_blocks(c->cmax > c->no3 ? c->cmax : c->no3);
  c->partial = P.take<double>(B * nred);
  c->prior = P.take<double>(B);
  c->data = P.take<double>(B);
}

void init_sizes(pmr_ctx* c, const pmr_config* cfg) {
  c->cfg = *cfg;
  c->B = cfg->batch;
  c->np = cfg->n_part;
  c->nm = cfg->n_mesh;
  c->no = cfg->n_out;
  c->n = cfg->n_steps;
  c->H = cfg->loss_kind == PMR_LOSS_LOGNORMAL && cfg->halo_model == PMR_HALO_SINGLE
             ? cfg->mlp_hidden
             : 0;
  c->k = cfg->ckpt_every >= cfg->n_steps ? 0 : cfg->ckpt_every;
  c->np3 = (size_t)c->np * c->np * c->np;
  c->nm3 = (size_t)c->nm * c->nm * c->nm;
  c->no3 = (size_t)c->no * c->no * c->no;
  c->cp = (size_t)c->np * c->np * (c->np / 2 + 1);
  c->cm = (size_t)c->nm * c->nm * (c->nm / 2 + 1);
  c->co = (size_t)c->no * c->no * (c->no / 2 + 1);
  c->sp = (size_t)c->np * c->np * spec_pitch(c->np);
  c->sm = (size_t)c->nm * c->nm * spec_pitch(c->nm);
  c->so = (size_t)c->no * c->no * spec_pitch(c->no);
  c->cmax = c->sp > c->sm ? c->sp : c->sm;
  if (c->so > c->cmax) c->cmax = c->so;
  c->log_np3 = ilog2(c->np3);
  c->log_nm = ilog2((size_t)c->nm);
  c->log_no = ilog2((size_t)c->no);
  if (c->k == 0) {
    c->n_xslots = c->n + 1;
    c->n_fslots = c->n;
    c->n_ck = 0;
  } else {
    c->n_xslots = c->k;  // ring slots 0..k-1 (segment starts live in the checkpoints)
    c->n_fslots = c->k;
    c->n_ck = (c->n + c->k - 1) / c->k;
  }
  c->mass_m = (float)std::pow((double)c->nm / c->np, 3);
  c->mass_o = (float)std::pow((double)c->no / c->np, 3);
}

void init_factors(pmr_ctx* c) {
  Cosmo cos{c->cfg.omega_m};
  const int n = c->n;
  std::vector<double> a(n + 1), D(n + 1), Gp(n + 1), Gph(n);
  for (int i = 0; i <= n; ++i) {
    a[i] = c->cfg.a0 + (c->cfg.a1 - c->cfg.a0) * (double)i / (double)n;
    D[i] = cos.D(a[i]);
    Gp[i] = cos.Gp(a[i]);
  }
  for (int i = 0; i < n; ++i) Gph[i] = cos.Gp(0.5 * (a[i] + a[i + 1]));
  c->kick.resize(n);
  c->drift.resize(n);
  for (int i = 0; i < n; ++i) {
    const double glo = i == 0 ? Gp[0] : Gph[i - 1];
    c->kick[i] = (Gph[i] - glo) / D[i];
    c->drift[i] = (D[i + 1] - D[i]) / Gph[i];
  }
  c->D0 = D[0];
  c->Gp0 = Gp[0];
}

int check(pmr_ctx* c) {
  if (c->status != PMR_OK) return c->status;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) c->status = PMR_E_HIP;
  return c->status;
}

// Records a (start, stop) event pair around the launches of the profiled kernel class on
// the context stream; `bytes` are the launch's algorithmic bytes.
struct ProfScope {
  pmr_ctx* c;
  bool on;
  ProfScope(pmr_ctx* ctx, int cls, double bytes) : c(ctx), on(false) {
    if (c->prof_class == cls && c->prof_used + 2 <= c->prof_ev.size()) {
      on = true;
      HIPC(c, hipEventRecord(c->prof_ev[c->prof_used], c->stream));
      c->prof_bytes += bytes;
    }
  }
  ~ProfScope() {
    if (on) {
      HIPC(c, hipEventRecord(c->prof_ev[c->prof_used + 1], c->stream));
      c->prof_used += 2;
    }
  }
};

// ---------------------------------------------------------------- pass helpers
FieldMap fmap(int fpi, size_t item_stride, size_t comp_stride, size_t pitch = 0) {
  FieldMap m;
  m.fpi = fpi;
  m.item_stride = item_stride;
  m.comp_stride = comp_stride;
  m.pitch = pitch;
  return m;
}

PaintArgs paint_args(const uint32_t* keys, const Vec3* frac, const Vec3* val,
                     const uint32_t* rows, int nm, float mass, float bias) {
  PaintArgs a{};
  a.keys = keys;
  a.frac = frac;
  a.val = val;
  a.row_start = rows;
  a.nm = nm;
  a.log_nm = (int)ilog2((size_t)nm);
  a.mass = mass;
  a.bias = bias;
  return a;
}

XPassArgs xargs(pmr_ctx* c, int n) {
  XPassArgs a;
  std::memset(&a, 0, sizeof(a));
  a.n = n;
  a.batch = c->B;
  a.box = c->cfg.box;
  a.R1 = c->cfg.R1;
  a.R2 = c->cfg.R2;
  a.params = c->params;
  a.in_pitch = a.out_pitch = spec_pitch(n);
  return a;
}

size_t cplx(int n) { return (size_t)n * n * (n / 2 + 1); }

// Real fields [B][ncomp][n^3] -> spectra in cB [B][3][cmax] (components 0..ncomp-1),
// completing the z and y passes; the x pass is fused with the caller's operator.
void r2c_zy(pmr_ctx* c, int n, int ncomp, const float* in, size_t in_item_stride,
            size_t in_comp_stride, const float* in2, float a1, float a2, const double* scale,
            float2* out, size_t out_item_stride, size_t out_comp_stride) {
  const int fields = c->B * ncomp;
  const double n3 = (double)n * n * n, cn = (double)n * n * (n / 2 + 1);
  {
    ProfScope ps(c, PMR_PROF_ZPASS, fields * ((in2 ? 8.0 : 4.0) * n3 + 8.0 * cn));
    launch_zpass_r2c(n, fields, in, fmap(ncomp, in_item_stride, in_comp_stride), in2, a1, a2,
                     scale, out, fmap(ncomp, out_item_stride, out_comp_stride, spec_pitch(n)),
                     c->stream);
  }
  {
    ProfScope ps(c, PMR_PROF_YPASS, fields * 16.0 * cn);
    launch_ypass(n, fields, out, fmap(ncomp, out_item_stride, out_comp_stride, spec_pitch(n)), false,
                 c->stream);
  }
}

// Spectra after the x pass -> real fields: inverse y, then c2r along z (with optional add).
void c2r_yz(pmr_ctx* c, int n, int ncomp, float2* in, size_t in_item_stride, size_t in_comp_stride,
            float* out, size_t out_item_stride, size_t out_comp_stride, const float* add) {
  const int fields = c->B * ncomp;
  const double n3 = (double)n * n * n, cn = (double)n * n * (n / 2 + 1);
  {
    ProfScope ps(c, PMR_PROF_YPASS, fields * 16.0 * cn);
    launch_ypass(n, fields, in, fmap(ncomp, in_item_stride, in_comp_stride, spec_pitch(n)), true,
                 c->stream);
  }
  {
    ProfScope ps(c, PMR_PROF_ZPASS, fields * (8.0 * cn + (add ? 8.0 : 4.0) * n3));
    launch_zpass_c2r(n, fields, in, fmap(ncomp, in_item_stride, in_comp_stride, spec_pitch(n)), out,
                     fmap(ncomp, out_item_stride, out_comp_stride), add, c->stream);
  }
}

// The kz windows of a transform on an n^3 mesh: one window of the whole half spectrum, or
// consecutive slabs of fft_slab_columns(n) columns.
std::vector<KzWin> kz_windows(int n) {
  const int w = fft_slab_columns(n), nh = n / 2 + 1;
  std::vector<KzWin> v;
  if (w <= 0) {
    v.push_back(KzWin{});
    return v;
  }
  for (int lo = 0; lo < nh; lo += w) v.push_back(KzWin{lo, lo + w < nh ? lo + w : nh});
  return v;
}

// Share of the half spectrum's columns in a window (for the algorithmic bytes of a launch).
double window_share(int n, const KzWin& win) {
  const int nh = n / 2 + 1;
  const int hi = win.hi > 0 && win.hi < nh ? win.hi : nh;
  return (double)(hi - win.lo) / nh;
}

// Gaussian smoothing of a real field [B][n^3] on R (per item, params[param_index]).
void smooth(pmr_ctx* c, int n, const float* in, int param_index, float* out, const float* add,
            const double* scale = nullptr, float a1 = 1.f) {
  const size_t n3 = (size_t)n * n * n, cn = (size_t)n * n * spec_pitch(n);
  r2c_zy(c, n, 1, in, n3, 0, nullptr, a1, 0.f, scale, c->cA, cn, 0);
  XPassArgs a = xargs(c, n);
  a.n_in = 1;
  a.n_out = 1;
  a.in[0] = c->cA;
  a.out[0] = c->cB;
  a.in_item_stride = cn;
  a.out_item_stride = cn;
  a.param_index = param_index;
  launch_xpass(XOP_GAUSS, a, c->stream);
  c2r_yz(c, n, 1, c->cB, cn, 0, out, n3, 0, add);
}

// ---------------------------------------------------------------- PM pieces
// Second-order LPT (Sec. 3 starts from 2LPT): the second-order growth is D2 = -(3/7) D^2
// (the Einstein-de Sitter ratio), so x0 gains (3/7) D0^2 Psi2 and p0 gains (6/7) D0 Gp0 Psi2.
constexpr double kLpt2 = 3.0 / 7.0;

// phi_ab = irfft(k_a k_b / k^2 P s) (two Hessian passes of three pairs), the source S, and
// Psi2 = irfft(i k / k^2 rfft(S)) into psi2.
void lpt2_forward(pmr_ctx* c) {
  const size_t cp = c->sp, np3 = c->np3;
  for (int set = 0; set < 2; ++set) {
    XPassArgs a = xargs(c, c->np);
    a.n_in = 1;
    a.n_out = 3;
    a.in[0] = c->ps;  // projected modes, standard layout
    for (int q = 0; q < 3; ++q) a.out[q] = c->cB + q * cp;
    a.in_item_stride = c->cp;
    a.in_pitch = (size_t)(c->np / 2 + 1);
    a.out_item_stride = 3 * cp;
    a.param_index = set;
    launch_xpass(XOP_HESS, a, c->stream);
    c2r_yz(c, c->np, 3, c->cB, 3 * cp, cp, c->phi + set * 3 * np3, 6 * np3, np3, nullptr);
  }
  launch_lpt2_source(c->phi, c->B, c->log_np3, c->psi2, 3 * np3, c->stream);
  r2c_zy(c, c->np, 1, c->psi2, 3 * np3, 0, nullptr, 1.f, 0.f, nullptr, c->cA, cp, 0);
  XPassArgs a = xargs(c, c->np);
  a.n_in = 1;
  a.n_out = 3;
  a.in[0] = c->cA;
  for (int q = 0; q < 3; ++q) a.out[q] = c->cB + q * cp;
  a.in_item_stride = cp;
  a.out_item_stride = 3 * cp;
  launch_xpass(XOP_FORCE, a, c->stream);
  c2r_yz(c, c->np, 3, c->cB, 3 * cp, cp, c->psi2, 3 * np3, np3, nullptr);
}

// Adds the second-order part of the gradient: Psi2_bar = (3/7) D0^2 x_bar + (6/7) D0 Gp0 p_bar,
// S_bar = sum_a irfft(conj(i k_a / k^2) rfft(Psi2_bar_a)), phi_bar from S_bar, and
// G += w(kz) sum_ab k_a k_b / k^2 rfft(phi_bar_ab) / n^3.
void lpt2_adjoint(pmr_ctx* c, float2* grad) {
  const size_t cp = c->sp, np3 = c->np3;
  r2c_zy(c, c->np, 3, c->xbar, 3 * np3, np3, c->pbar, (float)(kLpt2 * c->D0 * c->D0),
         (float)(2.0 * kLpt2 * c->D0 * c->Gp0), nullptr, c->cB, 3 * cp, cp);
  {
    XPassArgs a = xargs(c, c->np);
    a.n_in = 3;
    a.n_out = 1;
    for (int q = 0; q < 3; ++q) a.in[q] = c->cB + q * cp;
    a.out[0] = c->cA;
    a.in_item_stride = 3 * cp;
    a.out_item_stride = cp;
    launch_xpass(XOP_FORCE_ADJ, a, c->stream);
  }
  c2r_yz(c, c->np, 1, c->cA, cp, 0, c->psi2, 3 * np3, 0, nullptr);
  launch_lpt2_phi_bar(c->phi, c->psi2, 3 * np3, c->B, c->log_np3, c->phibar, c->stream);
  for (int set = 0; set < 2; ++set) {
    r2c_zy(c, c->np, 3, c->phibar + set * 3 * np3, 6 * np3, np3, nullptr, 1.f, 0.f, nullptr,
           c->cB, 3 * cp, cp);
    XPassArgs a = xargs(c, c->np);
    a.n_in = 3;
    a.n_out = 1;
    for (int q = 0; q < 3; ++q) a.in[q] = c->cB + q * cp;
    a.out[0] = grad;  // standard layout
    a.in_item_stride = 3 * cp;
    a.out_item_stride = c->cp;
    a.out_pitch = (size_t)(c->np / 2 + 1);
    a.param_index = set;
    launch_xpass(XOP_HESS_ADJ, a, c->stream);
  }
}

double* xslot(pmr_ctx* c, int s) { return c->xs + (size_t)s * c->B * 3 * c->np3; }
// Where x_i lives: with checkpointing, the positions at the start of a segment (i = j k < n)
// are the checkpoint j itself (the kick and drift before it write them there, recomputation
// reads them in place), the others a ring slot i mod k (x_n in slot 0 when k divides n);
// without, slot i.
double* xpos(pmr_ctx* c, int i) {
  if (c->k == 0) return xslot(c, i);
  if (i % c->k == 0 && i < c->n) return c->ckx + (size_t)(i / c->k) * c->B * 3 * c->np3;
  return xslot(c, i % c->k);
}
// The checkpointed momenta of segment j (the momenta at the start of step j k).
float* ckpt_p(pmr_ctx* c, int j) { return c->ckp + (size_t)j * c->B * 3 * c->np3; }
Vec3* fslot(pmr_ctx* c, int s) { return c->F + (size_t)s * c->B * c->nm3; }
uint32_t* idslot(pmr_ctx* c, int s) { return c->ids + (size_t)s * c->B * c->np3; }
uint32_t* keyslot(pmr_ctx* c, int s) { return c->skeys + (size_t)s * c->B * c->np3; }
Vec3* fracslot(pmr_ctx* c, int s) { return c->frac + (size_t)s * c->B * c->np3; }
uint32_t* invslot(pmr_ctx* c, int s) {
  return direct_sorted_values(c) ? c->inv + (size_t)s * c->B * c->np3 : nullptr;
}
uint32_t* rowslot(pmr_ctx* c, int s) { return c->rows + (size_t)s * (c->B * c->nm * c->nm + 1); }
int fs_of(pmr_ctx* c, int i) { return c->k == 0 ? i : i % c->k; }

// One forward PM step i: sort x_i, paint, force, kick + drift (keys of x_{i+1} emitted on
// the force mesh, or on the output mesh after the last step). `order`: the sorted ids of
// step i - 1 where its slot still holds them (the sort visits the particles in that order,
// which only makes it faster), else nullptr.
// `p_in`: the momenta before step i's kick when they are not in c->p (the checkpoint a
// recomputed segment starts from).
void pm_step(pmr_ctx* c, int i, bool advance = true, const uint32_t* order = nullptr,
             const float* p_in = nullptr) {
  const int B = c->B;
  const int total = (int)(B * c->np3);
  const int fsl = fs_of(c, i);
  double* x = xpos(c, i);
  double* xn = xpos(c, i + 1);
  {
    ProfScope ps(c, PMR_PROF_SORT, 0.0);
    launch_cell_sort(c->keys, order, total, c->log_nm, (size_t)B * c->nm * c->nm, keyslot(c, fsl),
                     idslot(c, fsl), rowslot(c, fsl), c->sort_scratch, c->frac_id,
                     fracslot(c, fsl), invslot(c, fsl), c->stream);
  }
  const size_t cm = c->sm;
  const FieldMap dm = fmap(1, cm, 0, spec_pitch(c->nm));
  {
    // density contrast painted and z-transformed in one pass (the real mesh stays in LDS)
    ProfScope ps(c, PMR_PROF_PAINT, 24.0 * B * c->np3 + 8.0 * B * c->cm);
    launch_paint_r2c(c->nm, 1, paint_args(keyslot(c, fsl), fracslot(c, fsl), nullptr,
                                          rowslot(c, fsl), c->nm, c->mass_m, 1.f),
                     B, c->cA, dm, c->stream);
  }
  // y forward; x pass: the x component i k_x / k^2 and the potential 1 / k^2 of the
  // density; y inverse of the x component, and of the potential into its y and z
  // derivatives (components 1 and 2). Window by window of kz columns when slabs are on, so
  // that each window's spectra stay in the memory-side cache between the passes.
  const FieldMap fm3 = fmap(3, 3 * cm, cm, spec_pitch(c->nm));
  const FieldMap fc0 = fmap(1, 3 * cm, 0, spec_pitch(c->nm));  // component 0 of each item
  for (const KzWin& win : kz_windows(c->nm)) {
    const double part = window_share(c->nm, win);
    {
      ProfScope ps(c, PMR_PROF_YPASS, part * 16.0 * B * c->cm);
      launch_ypass(c->nm, B, c->cA, dm, false, c->stream, win);
    }
    XPassArgs a = xargs(c, c->nm);
    a.n_in = 1;
    a.n_out = 2;
    a.in[0] = c->cA;
    a.out[0] = c->cB;
    a.out[1] = c->cB + cm;
    a.in_item_stride = cm;
    a.out_item_stride = 3 * cm;
    a.kz_lo = win.lo;
    a.kz_hi = win.hi;
    {
      ProfScope ps(c, PMR_PROF_XPASS_FORCE, part * 24.0 * B * c->cm);
      launch_xpass(XOP_FORCE_X, a, c->stream);
    }
    {
      ProfScope ps(c, PMR_PROF_YPASS, part * 16.0 * B * c->cm);
      launch_ypass(c->nm, B, c->cB, fc0, true, c->stream, win);
    }
    XPassArgs y = xargs(c, c->nm);
    y.n_in = 1;
    y.n_out = 2;
    y.in[0] = c->cB + cm;
    y.out[0] = c->cB + cm;
    y.out[1] = c->cB + 2 * cm;
    y.in_item_stride = y.out_item_stride = 3 * cm;
    y.kz_lo = win.lo;
    y.kz_hi = win.hi;
    {
      ProfScope ps(c, PMR_PROF_YPASS, part * 24.0 * B * c->cm);
      launch_xpass(XOP_YGRAD, y, c->stream);
    }
  }
  Vec3* F = fslot(c, fsl);
  {
    ProfScope ps(c, PMR_PROF_ZPASS, 3 * 8.0 * B * c->cm + B * 12.0 * c->nm3);
    launch_zpass_c2r3(c->nm, c->B, c->cB, fm3, F, c->nm3, c->stream);
  }
  if (!advance) return;  // (x, p) of step i + 1 already held elsewhere (a checkpoint)
  const int key_nm = (i == c->n - 1) ? c->no : c->nm;
  {
    // compulsory: x (FP64) and p read and written per particle, the three force channels
    // per cell (the keys and fractions of the next sort count in time only)
    ProfScope ps(c, PMR_PROF_KICK_DRIFT, 72.0 * B * c->np3 + 12.0 * B * c->nm3);
    // the momenta that start the next segment also go to its checkpoint
    float* pck = (c->k > 0 && (i + 1) % c->k == 0 && i + 1 < c->n) ? ckpt_p(c, (i + 1) / c->k)
                                                                      : nullptr;
    launch_kick_drift(x, xn, p_in, c->p, pck, F, c->keys, c->frac_id, B, c->log_np3, c->nm,
                      c->cfg.box, (float)c->kick[i], c->drift[i], key_nm, c->stream);
  }
}

// Run forward steps [i0, i1) (positions x_{i0} in place, momenta in c->p); the checkpoints
// are written by the steps themselves (xpos, ckpt_p).
void pm_run(pmr_ctx* c, int i0, int i1) {
  for (int i = i0; i < i1; ++i)
    pm_step(c, i, true, i > 0 ? idslot(c, fs_of(c, i - 1)) : nullptr);
}


// x_data = log(G_Rmass * M_target + M0), enqueued as soon as both target and loss
// parameters are known, so that captured forward passes never depend on host state.
void refresh_xd(pmr_ctx* c) {
  if (c->cfg.loss_kind != PMR_LOSS_LOGNORMAL || !c->have_target || !c->have_loss) return;
  smooth(c, c->no, c->target, 3, c->ob, nullptr);
  launch_target_x(c->ob, c->no3, c->B, c->params, c->xd, c->stream);
  if (c->noise_k > 0)
    launch_noise_fields(c->ob, (size_t)c->B * c->no3, c->noise_tab, c->noise_k, c->noise_mu,
                        c->noise_w, c->stream);
  c->xd_dirty = 0;
}

}  // namespace

// ================================================================ C ABI
extern "C" {

size_t pmr_workspace_bytes(const pmr_config* cfg) {
  if (validate(cfg) != PMR_OK) return 0;
  pmr_ctx c;
  init_sizes(&c, cfg);
  Plan P{nullptr, 0};
  plan(&c, P);
  return P.off;
}

int pmr_create(const pmr_config* cfg, void* workspace, size_t bytes, void* stream, pmr_ctx** out) {
  if (!out) return PMR_E_INVALID;
  *out = nullptr;
  int st = validate(cfg);
  if (st != PMR_OK) return st;
  if (!workspace || ((uintptr_t)workspace & 255)) return PMR_E_WORKSPACE;
  if (bytes < pmr_workspace_bytes(cfg)) return PMR_E_WORKSPACE;
  pmr_ctx* c = new (std::nothrow) pmr_ctx();
  if (!c) return PMR_E_INVALID;
  init_sizes(c, cfg);
  c->stream = (hipStream_t)stream;
  c->ws = (char*)workspace;
  c->ws_bytes = bytes;
  c->status = PMR_OK;
  Plan P{c->ws, 0};
  plan(c, P);
  init_factors(c);
  *out = c;
  return PMR_OK;
}

int pmr_set_stream(pmr_ctx* c, void* stream) {
  if (!c) return PMR_E_INVALID;
  c->stream = (hipStream_t)stream;
  return PMR_OK;
}

int pmr_destroy(pmr_ctx* c) {
  if (c)
    for (hipEvent_t e : c->prof_ev) (void)hipEventDestroy(e);
  delete c;
  return PMR_OK;
}

int pmr_set_prior(pmr_ctx* c, const float* inv_var) {
  if (!c || !inv_var) return PMR_E_INVALID;
  HIPC(c, hipMemcpyAsync(c->inv_var, inv_var, c->cp * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
  c->have_prior = 1;
  return check(c);
}

int pmr_set_mlp(pmr_ctx* c, const float* W1, const float* b1, const float* W2, const float* b2,
                const float* W3, const float* b3) {
  if (!c || !W1 || !b1 || !W2 || !b2 || !W3 || !b3) return PMR_E_INVALID;
  if (c->H == 0) return PMR_E_STATE;
  const int H = c->H;
  float* w = c->mlp_w;
  const size_t f = sizeof(float);
  HIPC(c, hipMemcpyAsync(w, W1, 3 * H * f, hipMemcpyDeviceToDevice, c->stream));
  HIPC(c, hipMemcpyAsync(w + 3 * H, b1, H * f, hipMemcpyDeviceToDevice, c->stream));
  HIPC(c, hipMemcpyAsync(w + 4 * H, W2, (size_t)H * H * f, hipMemcpyDeviceToDevice, c->stream));
  HIPC(c, hipMemcpyAsync(w + 4 * H + H * H, b2, H * f, hipMemcpyDeviceToDevice, c->stream));
  HIPC(c, hipMemcpyAsync(w + 5 * H + H * H, W3, H * f, hipMemcpyDeviceToDevice, c->stream));
  HIPC(c, hipMemcpyAsync(w + 6 * H + H * H, b3, f, hipMemcpyDeviceToDevice, c->stream));
  if (c->cfg.precision == PMR_MIXED && launch_mlp_prepare_bf16(H, w, c->stream) != 0)
    return PMR_E_SHAPE;
  c->have_mlp = 1;
  return check(c);
}

int pmr_set_halo_nets(pmr_ctx* c, const float* nnp, const float* nnm) {
  if (!c || !nnp || !nnm) return PMR_E_INVALID;
  if (c->cfg.halo_model != PMR_HALO_TWO) return PMR_E_STATE;
  launch_halo2_prepare(nnp, nnm, c->halo2_w, c->stream);
  c->have_mlp = 1;
  return check(c);
}

int pmr_set_target(pmr_ctx* c, const float* target) {
  if (!c || !target) return PMR_E_INVALID;
  HIPC(c, hipMemcpyAsync(c->target, target, c->B * c->no3 * sizeof(float), hipMemcpyDeviceToDevice,
                 c->stream));
  c->have_target = 1;
  c->xd_dirty = 1;
  refresh_xd(c);
  return check(c);
}

int pmr_set_noise_table(pmr_ctx* c, int n_nodes, const double* log_mass, const double* mu,
                        const double* sigma) {
  if (!c || n_nodes < 0 || n_nodes > NOISE_MAX) return PMR_E_INVALID;
  if (n_nodes > 0 && (!log_mass || !mu || !sigma)) return PMR_E_INVALID;
  std::vector<double> h(3 * NOISE_MAX, 0.0);
  for (int j = 0; j < n_nodes; ++j) {
    if (!std::isfinite(log_mass[j]) || !std::isfinite(mu[j]) || !(sigma[j] > 0) ||
        !std::isfinite(sigma[j]) || (j > 0 && !(log_mass[j] > log_mass[j - 1])))
      return PMR_E_INVALID;
    h[j] = log_mass[j];
    h[NOISE_MAX + j] = mu[j];
    h[2 * NOISE_MAX + j] = sigma[j];
  }
  // the table travels as kernel arguments: stream-ordered, no wait for the host
  launch_noise_table_store(h.data(), c->noise_tab, c->stream);
  c->noise_k = n_nodes;
  c->xd_dirty = 1;
  refresh_xd(c);
  return check(c);
}

static_assert(sizeof(pmr_loss_params) == PMR_LOSS_FIELDS * sizeof(double),
              "pmr_loss_params is read on the device as consecutive doubles");

int pmr_set_loss(pmr_ctx* c, const pmr_loss_params* prm) {
  if (!c || !prm) return PMR_E_INVALID;
  std::vector<double> h(NPRM * (size_t)c->B);
  for (int b = 0; b < c->B; ++b) {
    const pmr_loss_params& q = prm[b];
    if (!(q.sigma_N > 0) || !(q.M0 > 0 || c->cfg.loss_kind == PMR_LOSS_DENSITY_L2) ||
        !(q.R_mass >= 0) || !(q.R_sm >= 0) || !std::isfinite(q.mu) || !std::isfinite(q.prior_weight))
      return PMR_E_INVALID;
    if (c->cfg.halo_model == PMR_HALO_TWO && !(q.logistic_a > 0 && std::isfinite(q.logistic_a)))
      return PMR_E_INVALID;
    double* d = h.data() + NPRM * (size_t)b;
    d[0] = q.M0;
    d[1] = q.mu;
    d[2] = q.sigma_N;
    d[3] = q.R_mass;
    d[4] = q.R_sm;
    d[5] = q.prior_weight;
    d[6] = q.logistic_a;
    d[PRM_VALID] = 1.0;
  }
  // the values travel as kernel arguments: stream-ordered, no wait for the host
  launch_params_store(h.data(), c->B, c->params, c->stream);
  c->have_loss = 1;
  c->xd_dirty = 1;
  refresh_xd(c);
  return check(c);
}

int pmr_set_loss_device(pmr_ctx* c, const pmr_loss_params* params_device) {
  if (!c || !params_device) return PMR_E_INVALID;
  if (((uintptr_t)params_device & 7) != 0) return PMR_E_INVALID;
  launch_params_from_device((const double*)params_device, c->B,
                            c->cfg.loss_kind == PMR_LOSS_DENSITY_L2,
                            c->cfg.halo_model == PMR_HALO_TWO, c->params, c->stream);
  c->have_loss = 1;
  c->xd_dirty = 1;
  refresh_xd(c);
  return check(c);
}

long long pmr_forward_count(const pmr_ctx* c) { return c ? c->n_forward : PMR_E_INVALID; }

int pmr_forward(pmr_ctx* c, const void* modes, float* mass_out, double* loss_out) {
  if (!c || !modes || !loss_out) return PMR_E_INVALID;
  if (c->status != PMR_OK) return c->status;
  if (!c->have_prior || !c->have_target || !c->have_loss) return PMR_E_STATE;
  if (c->cfg.loss_kind == PMR_LOSS_LOGNORMAL && !c->have_mlp) return PMR_E_STATE;
  const int B = c->B;
  hipStream_t s = c->stream;
  // H0: projection and prior
  launch_project_prior((const float2*)modes, c->np, B, c->inv_var, c->ps, c->partial, c->prior, s);
  // data term of the target (log-normal): x_data = log(G_Rmass * M_t + M0)
  if (c->xd_dirty) refresh_xd(c);
  // H1: Zel'dovich displacement on the particle lattice
  {
    const size_t cp = c->sp;
    XPassArgs a = xargs(c, c->np);
    a.n_in = 1;
    a.n_out = 3;
    a.in[0] = c->ps;  // projected modes, standard layout
    for (int q = 0; q < 3; ++q) a.out[q] = c->cB + q * cp;
    a.in_item_stride = c->cp;
    a.in_pitch = (size_t)(c->np / 2 + 1);
    a.out_item_stride = 3 * cp;
    launch_xpass(XOP_ZA, a, s);
    c2r_yz(c, c->np, 3, c->cB, 3 * cp, cp, c->psi, 3 * c->np3, c->np3, nullptr);
    const bool second = c->cfg.ic_order == 2;
    if (second) lpt2_forward(c);
    const int key_nm = c->n == 0 ? c->no : c->nm;
    launch_za_init(c->psi, second ? c->psi2 : nullptr, B, c->np, c->log_np3, c->cfg.box,
                   0.5 * (c->cfg.box / c->nm), c->D0, (float)c->Gp0,
                   second ? kLpt2 * c->D0 * c->D0 : 0.0,
                   second ? (float)(2.0 * kLpt2 * c->D0 * c->Gp0) : 0.f, xpos(c, 0), c->p,
                   c->k > 0 ? ckpt_p(c, 0) : nullptr, c->keys, c->frac_id, key_nm, s);
  }
  // H2-H7: the PM steps
  pm_run(c, 0, c->n);
  // H8: final paint on the output mesh
  const int total = (int)(B * c->np3);
  {
    ProfScope ps(c, PMR_PROF_SORT, 0.0);
    launch_cell_sort(c->keys, idslot(c, fs_of(c, c->n - 1)), total, c->log_no,
                     (size_t)B * c->no * c->no, c->keys_sorted,
                     c->ids_o, c->rows_o, c->sort_scratch, c->frac_id, c->frac_o, nullptr, s);
  }
  launch_paint_mass(c->keys_sorted, c->frac_o, c->rows_o, B, c->no, c->mass_o, 1.f, c->delta_f, s);
  // H9-H11: halo model and likelihood
  if (c->cfg.loss_kind == PMR_LOSS_DENSITY_L2) {
    launch_sumsq(c->delta_f, c->target, c->no3, B, c->partial, c->data, s);
    if (mass_out)
      HIPC(c, hipMemcpyAsync(mass_out, c->delta_f, B * c->no3 * sizeof(float), hipMemcpyDeviceToDevice, s));
  } else {
    const size_t no3 = c->no3, co = c->so;
    r2c_zy(c, c->no, 1, c->delta_f, no3, 0, nullptr, 1.f, 0.f, nullptr, c->cA, co, 0);
    XPassArgs a = xargs(c, c->no);
    a.n_in = 1;
    a.n_out = 2;
    a.in[0] = c->cA;
    a.out[0] = c->cB;
    a.out[1] = c->cB + co;
    a.in_item_stride = co;
    a.out_item_stride = 3 * co;
    launch_xpass(XOP_GAUSS2, a, s);
    c2r_yz(c, c->no, 2, c->cB, 3 * co, co, c->dR, no3, (size_t)B * no3, nullptr);
    if (c->cfg.halo_model == PMR_HALO_TWO) {
      ProfScope ps(c, PMR_PROF_HALO2, 2.0 * HALO2_FWD_FMA * B * no3);
      launch_halo2_fwd(c->delta_f, c->dR, c->dR + (size_t)B * no3, c->log_no, (size_t)B * no3,
                       c->halo2_w, c->params, c->h2aux, c->h2sgn, c->mass, s);
    } else {
      const double Hd = c->H;
      ProfScope ps(c, PMR_PROF_NETWORK, 2.0 * (4.0 * Hd + Hd * Hd) * B * no3);
      const int rc = c->cfg.precision == PMR_MIXED
                         ? launch_mlp_fwd_mfma(c->H, c->delta_f, c->dR, c->dR + (size_t)B * no3,
                                               (size_t)B * no3, c->mlp_w, c->mass, s)
                         : launch_mlp_fwd(c->H, c->delta_f, c->dR, c->dR + (size_t)B * no3,
                                          (size_t)B * no3, c->mlp_w, c->mass, s);
      if (rc != 0) return PMR_E_SHAPE;
    }
    smooth(c, c->no, c->mass, 3, c->MR, nullptr);
    launch_residual(c->MR, c->xd, no3, B, c->params, c->noise_k ? c->noise_mu : nullptr,
                    c->noise_k ? c->noise_w : nullptr, c->r, s);
    smooth(c, c->no, c->r, 4, c->rs, nullptr);
    launch_sumsq(c->rs, nullptr, no3, B, c->partial, c->data, s);
    if (mass_out) HIPC(c, hipMemcpyAsync(mass_out, c->mass, B * no3 * sizeof(float), hipMemcpyDeviceToDevice, s));
  }
  launch_finalize_loss(c->prior, c->data, c->params, B, loss_out, s);
  c->fwd_done = 1;
  ++c->n_forward;
  const int st = check(c);
  if (st != PMR_OK || !c->check_finite) return st;
  std::vector<double> h(3 * (size_t)B);
  HIPC(c, hipMemcpyAsync(h.data(), loss_out, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPC(c, hipStreamSynchronize(s));
  if (c->status != PMR_OK) return c->status;
  for (double v : h)
    if (!std::isfinite(v)) return PMR_E_NONFINITE;
  return PMR_OK;
}

int pmr_set_check_finite(pmr_ctx* c, int on) {
  if (!c) return PMR_E_INVALID;
  c->check_finite = on != 0;
  return PMR_OK;
}

int pmr_adjoint(pmr_ctx* c, const double* loss_bar, const float* mass_bar, void* grad) {
  if (!c || !loss_bar || !grad) return PMR_E_INVALID;
  if (c->status != PMR_OK) return c->status;
  if (!c->fwd_done) return PMR_E_STATE;
  const int B = c->B;
  hipStream_t s = c->stream;
  const size_t no3 = c->no3, co = c->so;
  float* dbar_f = c->ob + 3 * (size_t)B * no3;
  // H12-H13: likelihood, network and feature adjoints -> dbar_f
  if (c->cfg.loss_kind == PMR_LOSS_DENSITY_L2) {
    launch_l2_adj(c->delta_f, c->target, no3, B, loss_bar, mass_bar, dbar_f, s);
  } else {
    float* o0 = c->ob;
    float* o1 = c->ob + (size_t)B * no3;
    float* o2 = c->ob + 2 * (size_t)B * no3;
    smooth(c, c->no, c->rs, 4, o0, nullptr, loss_bar, 2.f);  // rbar = G_Rsm (2 loss_bar r_s)
    launch_mrbar(o0, c->MR, no3, B, c->params, c->noise_k ? c->noise_w : nullptr, o1,
                 s);  // MRbar
    smooth(c, c->no, o1, 3, o2, mass_bar);                   // Mbar (+ mass_bar)
    if (c->cfg.halo_model == PMR_HALO_TWO) {
      {
        ProfScope ps(c, PMR_PROF_HALO2, 2.0 * HALO2_BWD_FMA * B * no3);
        launch_halo2_bwd(c->delta_f, c->dR, c->dR + (size_t)B * no3, c->log_no, (size_t)B * no3,
                         c->halo2_w, c->params, o2, c->h2aux, c->h2sgn, c->u2, o0, o1, dbar_f,
                         s);
      }
      // compulsory: u (81 floats) read, three adjoint fields read and written, per voxel
      ProfScope ps(c, PMR_PROF_HALO2_STENCIL, (81.0 * 4 + 24.0) * B * no3);
      launch_halo2_stencil_adj(c->u2, c->log_no, (size_t)B * no3, o0, o1, dbar_f, s);
    } else {
      const double Hd = c->H;
      ProfScope ps(c, PMR_PROF_NETWORK, 2.0 * (8.0 * Hd + 2.0 * Hd * Hd) * B * no3);
      if (c->cfg.precision == PMR_MIXED)
        launch_mlp_bwd_mfma(c->H, c->delta_f, c->dR, c->dR + (size_t)B * no3, (size_t)B * no3,
                            c->mlp_w, o2, o0, o1, dbar_f, s);
      else
        launch_mlp_bwd(c->H, c->delta_f, c->dR, c->dR + (size_t)B * no3, (size_t)B * no3,
                       c->mlp_w, o2, o0, o1, dbar_f, s);
    }
    // g0 -> o0, g12 -> o1, g2 -> dbar_f (temporarily); feature adjoint:
    // dbar_f = g0 + irfft(G1 rfft(g12) - G2 rfft(g2))
    const size_t po = spec_pitch(c->no);
    launch_zpass_r2c(c->no, B, o1, fmap(1, no3, 0), nullptr, 1.f, 0.f, nullptr, c->cB,
                     fmap(1, 3 * co, 0, po), s);
    launch_zpass_r2c(c->no, B, dbar_f, fmap(1, no3, 0), nullptr, 1.f, 0.f, nullptr, c->cB + co,
                     fmap(1, 3 * co, 0, po), s);
    launch_ypass(c->no, 2 * B, c->cB, fmap(2, 3 * co, co, po), false, s);
    XPassArgs a = xargs(c, c->no);
    a.n_in = 2;
    a.n_out = 1;
    a.in[0] = c->cB;
    a.in[1] = c->cB + co;
    a.out[0] = c->cA;
    a.in_item_stride = 3 * co;
    a.out_item_stride = co;
    launch_xpass(XOP_FEAT_ADJ, a, s);
    c2r_yz(c, c->no, 1, c->cA, co, 0, dbar_f, no3, 0, o0);
  }
  // H14: final-paint adjoint -> xbar_n, pbar = 0
  // (the sort of the final positions on the output mesh is still held from the forward)
  launch_adjoint_positions(c->keys_sorted, c->frac_o, nullptr, c->ids_o, nullptr, dbar_f,
                           (int)(B * c->np3), c->no, c->cfg.box, c->mass_o, c->gpos, s);
  // the paint values of step n - 1, in its sort order when they go there directly (its
  // slot is held)
  bool vsorted = direct_sorted_values(c);  // c->vstream holds step i's values in sort order
  launch_adjoint_update(c->xbar, c->pbar, c->gpos, B, c->log_np3, 0.f, 0.f, 1,
                        vsorted ? c->vstream : c->vid, (float)c->kick[c->n - 1],
                        (float)c->drift[c->n - 1], invslot(c, fs_of(c, c->n - 1)), s);
  // H15: reverse PM steps (recomputing segments from checkpoints when needed)
  const size_t cm = c->sm;
  const double scale_m = (double)c->nm / c->cfg.box;
  int resident_lo = c->k == 0 ? 0 : ((c->n - 1) / c->k) * c->k;  // first step held in slots
  for (int i = c->n - 1; i >= 0; --i) {
    if (c->k > 0 && i < resident_lo) {
      const int j = (i / c->k) * c->k;
      // the segment starts from its checkpoint, read in place (x) and as the first kick's
      // input (p)
      launch_keys(xpos(c, j), c->log_np3, (int)(B * c->np3), scale_m, c->nm, c->keys,
                  c->frac_id, s);
      const int end = j + c->k < c->n ? j + c->k : c->n;
      // the adjoint of steps j .. end-1 needs x, the sort and F of each step, not the
      // positions the last kick and drift would produce (the next checkpoint)
      for (int q = j; q < end; ++q)
        pm_step(c, q, q + 1 < end, q > j ? idslot(c, fs_of(c, q - 1)) : nullptr,
                q == j ? ckpt_p(c, j / c->k) : nullptr);
      resident_lo = j;
      // the slots no longer hold the last segment: another adjoint needs a new forward
      c->fwd_done = 0;
    }
    const int fsl = fs_of(c, i);
    const float K = (float)c->kick[i], Dr = (float)c->drift[i];
    if (!vsorted) launch_stream_gather(idslot(c, fsl), c->vid, (int)(B * c->np3), c->vstream, s);
    const FieldMap fm3 = fmap(3, 3 * cm, cm, spec_pitch(c->nm));
    const FieldMap fc0 = fmap(1, 3 * cm, 0, spec_pitch(c->nm));  // component 0 of each item
    {
      // adjoint paint of the three force channels, z-transformed in the same pass
      ProfScope ps(c, PMR_PROF_PAINT3, (24.0 + 12.0) * B * c->np3 + 24.0 * B * c->cm);
      launch_paint_r2c(c->nm, 3, paint_args(keyslot(c, fsl), fracslot(c, fsl), c->vstream,
                                            rowslot(c, fsl), c->nm, 1.f, 0.f),
                       B, c->cB, fm3, s);
    }
    const FieldMap dm1 = fmap(1, cm, 0, spec_pitch(c->nm));
    for (const KzWin& win : kz_windows(c->nm)) {
      const double part = window_share(c->nm, win);
      {
        ProfScope ps(c, PMR_PROF_YPASS, part * 16.0 * B * c->cm);
        launch_ypass(c->nm, B, c->cB, fc0, false, s, win);
      }
      // components 1 and 2 forward along y, combined as conj(i k_y) Y + conj(i k_z) Z into
      // component 1
      XPassArgs y = xargs(c, c->nm);
      y.n_in = 2;
      y.n_out = 1;
      y.in[0] = c->cB + cm;
      y.in[1] = c->cB + 2 * cm;
      y.out[0] = c->cB + cm;
      y.in_item_stride = y.out_item_stride = 3 * cm;
      y.kz_lo = win.lo;
      y.kz_hi = win.hi;
      {
        ProfScope ps(c, PMR_PROF_YPASS, part * 24.0 * B * c->cm);
        launch_xpass(XOP_YGRAD_ADJ, y, s);
      }
      XPassArgs a = xargs(c, c->nm);
      a.n_in = 2;
      a.n_out = 1;
      a.in[0] = c->cB;
      a.in[1] = c->cB + cm;
      a.out[0] = c->cA;
      a.in_item_stride = 3 * cm;
      a.out_item_stride = cm;
      a.kz_lo = win.lo;
      a.kz_hi = win.hi;
      {
        ProfScope ps(c, PMR_PROF_XPASS_FORCE_ADJ, part * 24.0 * B * c->cm);
        launch_xpass(XOP_FORCE_X_ADJ, a, s);
      }
      {
        ProfScope ps(c, PMR_PROF_YPASS, part * 16.0 * B * c->cm);
        launch_ypass(c->nm, B, c->cA, dm1, true, s, win);
      }
    }
    {
      ProfScope ps(c, PMR_PROF_ZPASS, B * (8.0 * c->cm + 4.0 * c->nm3));
      launch_zpass_c2r(c->nm, B, c->cA, dm1, c->dbar, fmap(1, c->nm3, 0), nullptr, s);
    }
    {
      // compulsory: position (FP64), Fbar in and g out per particle; F and dbar per cell
      ProfScope ps(c, PMR_PROF_ADJ_GATHER, 48.0 * B * c->np3 + 16.0 * B * c->nm3);
      launch_adjoint_positions(keyslot(c, fsl), fracslot(c, fsl), c->vstream, idslot(c, fsl),
                               fslot(c, fsl), c->dbar, (int)(B * c->np3), c->nm, c->cfg.box,
                               c->mass_m, c->gpos, s);
    }
    {
      // xbar, pbar and g in; xbar, pbar and the next paint values out
      ProfScope ps(c, PMR_PROF_ADJ_UPDATE, (i > 0 ? 72.0 : 60.0) * B * c->np3);
      // step i - 1's paint values: into its sort order when that sort is held, else in id
      // order for a gather after its segment has been recomputed
      const bool next_sorted = direct_sorted_values(c) && i > 0 && i - 1 >= resident_lo;
      launch_adjoint_update(c->xbar, c->pbar, c->gpos, B, c->log_np3, K, Dr, 0,
                            i == 0 ? nullptr : next_sorted ? c->vstream : c->vid,
                            i > 0 ? (float)c->kick[i - 1] : 0.f,
                            i > 0 ? (float)c->drift[i - 1] : 0.f,
                            next_sorted ? invslot(c, fs_of(c, i - 1)) : nullptr, s);
      vsorted = next_sorted;
    }
  }
  // H16: Zel'dovich adjoint and gradient assembly (with the prior)
  {
    const size_t cp = c->sp;
    r2c_zy(c, c->np, 3, c->xbar, 3 * c->np3, c->np3, c->pbar, (float)c->D0, (float)c->Gp0, nullptr,
           c->cB, 3 * cp, cp);
    XPassArgs a = xargs(c, c->np);
    a.n_in = 3;
    a.n_out = 1;
    for (int q = 0; q < 3; ++q) a.in[q] = c->cB + q * cp;
    a.out[0] = (float2*)grad;  // standard layout, like proj_modes and the prior table
    a.in_item_stride = 3 * cp;
    a.out_item_stride = c->cp;
    a.out_pitch = (size_t)(c->np / 2 + 1);
    a.aux_item_stride = c->cp;
    a.proj_modes = c->ps;
    a.inv_var = c->inv_var;
    a.loss_bar = loss_bar;
    launch_xpass(XOP_ZA_ADJ, a, s);
    if (c->cfg.ic_order == 2) lpt2_adjoint(c, (float2*)grad);
  }
  return check(c);
}

int pmr_profile_begin(pmr_ctx* c, int kernel_class, int max_launches) {
  if (!c || kernel_class < 0 || max_launches < 0) return PMR_E_INVALID;
  const size_t need = 2 * (size_t)max_launches;
  while (c->prof_ev.size() < need) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return PMR_E_HIP;
    c->prof_ev.push_back(e);
  }
  c->prof_class = kernel_class;
  c->prof_used = 0;
  c->prof_bytes = 0.0;
  c->prof_open = false;
  return PMR_OK;
}

int pmr_profile_end(pmr_ctx* c, double* total_ms, long long* launches, double* alg_bytes) {
  if (!c || !total_ms || !launches || !alg_bytes) return PMR_E_INVALID;
  HIPC(c, hipStreamSynchronize(c->stream));
  double ms = 0.0;
  for (size_t i = 0; i + 1 < c->prof_used; i += 2) {
    float t = 0.f;
    HIPC(c, hipEventElapsedTime(&t, c->prof_ev[i], c->prof_ev[i + 1]));
    ms += t;
  }
  *total_ms = ms;
  *launches = (long long)(c->prof_used / 2);
  *alg_bytes = c->prof_bytes;
  c->prof_class = 0;
  c->prof_used = 0;
  c->prof_bytes = 0.0;
  return check(c);
}

const char* pmr_status_string(int st) {
  switch (st) {
    case PMR_OK: return "ok";
    case PMR_E_INVALID: return "invalid argument";
    case PMR_E_SHAPE: return "unsupported shape";
    case PMR_E_WORKSPACE: return "workspace too small or misaligned";
    case PMR_E_HIP: return "HIP runtime error";
    case PMR_E_NONFINITE: return "non-finite loss";
    case PMR_E_STATE: return "call out of order or missing inputs";
    default: return "unknown status";
  }
}

long long pmr_debug_copy(pmr_ctx* c, int what, int step, void* dst) {
  if (!c || !dst) return PMR_E_INVALID;
  const size_t B = c->B;
  const void* src = nullptr;
  size_t bytes = 0;
  switch (what) {
    case PMR_DBG_X: {
      if (step < 0 || step > c->n) return PMR_E_INVALID;
      if (c->k > 0 && step % c->k != 0) {
        // ring slots hold the last segment (checkpointed steps are always held)
        const int lo = ((c->n - 1) / c->k) * c->k;
        if (step < lo) return PMR_E_STATE;
      }
      src = xpos(c, step);
      bytes = B * 3 * c->np3 * sizeof(double);
      break;
    }
    case PMR_DBG_FORCE:
    case PMR_DBG_SORT_IDS: {
      if (step < 0 || step >= c->n) return PMR_E_INVALID;
      int sl;
      if (c->k == 0) sl = step;
      else {
        const int lo = ((c->n - 1) / c->k) * c->k;
        if (step < lo) return PMR_E_STATE;
        sl = step - lo;
      }
      if (what == PMR_DBG_FORCE) {
        src = fslot(c, sl);
        bytes = B * c->nm3 * sizeof(Vec3);
      } else {
        src = idslot(c, sl);
        bytes = B * c->np3 * sizeof(uint32_t);
      }
      break;
    }
    case PMR_DBG_DELTA_F: src = c->delta_f; bytes = B * c->no3 * sizeof(float); break;
    case PMR_DBG_FEATURES: src = c->dR; bytes = 2 * B * c->no3 * sizeof(float); break;
    case PMR_DBG_MASS_R: src = c->MR; bytes = B * c->no3 * sizeof(float); break;
    case PMR_DBG_RES_S: src = c->rs; bytes = B * c->no3 * sizeof(float); break;
    case PMR_DBG_XBAR0: src = c->xbar; bytes = B * 3 * c->np3 * sizeof(float); break;
    case PMR_DBG_PBAR0: src = c->pbar; bytes = B * 3 * c->np3 * sizeof(float); break;
    case PMR_DBG_DBAR_F: src = c->ob + 3 * B * c->no3; bytes = B * c->no3 * sizeof(float); break;
    default: return PMR_E_INVALID;
  }
  HIPC(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, c->stream));
  const int st = check(c);
  return st == PMR_OK ? (long long)bytes : st;
}

// ---------------------------------------------------------------- primitives
int pmr_fft_r2c(int n, int batch, const float* in, void* out, void* stream) {
  if (!in || !out || batch < 1) return PMR_E_INVALID;
  if (!pow2_in(n, 16, 512)) return PMR_E_SHAPE;
  hipStream_t s = (hipStream_t)stream;
  const size_t n3 = (size_t)n * n * n, cn = cplx(n);
  const size_t nh = (size_t)(n / 2 + 1);  // the caller's array has the standard pitch
  float2* o = (float2*)out;
  launch_zpass_r2c(n, batch, in, fmap(1, n3, 0), nullptr, 1.f, 0.f, nullptr, o, fmap(1, cn, 0, nh),
                   s);
  launch_ypass(n, batch, o, fmap(1, cn, 0, nh), false, s);
  XPassArgs a;
  std::memset(&a, 0, sizeof(a));
  a.n = n;
  a.batch = batch;
  a.n_in = a.n_out = 1;
  a.in[0] = o;
  a.out[0] = o;
  a.in_item_stride = a.out_item_stride = cn;
  a.in_pitch = a.out_pitch = nh;
  a.box = 1.0;
  launch_xpass(XOP_FWD, a, s);
  return hipGetLastError() == hipSuccess ? PMR_OK : PMR_E_HIP;
}

int pmr_fft_c2r(int n, int batch, void* inout, float* out, void* stream) {
  if (!inout || !out || batch < 1) return PMR_E_INVALID;
  if (!pow2_in(n, 16, 512)) return PMR_E_SHAPE;
  hipStream_t s = (hipStream_t)stream;
  const size_t n3 = (size_t)n * n * n, cn = cplx(n);
  const size_t nh = (size_t)(n / 2 + 1);
  float2* d = (float2*)inout;
  XPassArgs a;
  std::memset(&a, 0, sizeof(a));
  a.n = n;
  a.batch = batch;
  a.n_in = a.n_out = 1;
  a.in[0] = d;
  a.out[0] = d;
  a.in_item_stride = a.out_item_stride = cn;
  a.in_pitch = a.out_pitch = nh;
  a.box = 1.0;
  launch_xpass(XOP_INV, a, s);
  launch_ypass(n, batch, d, fmap(1, cn, 0, nh), true, s);
  launch_zpass_c2r(n, batch, d, fmap(1, cn, 0, nh), out, fmap(1, n3, 0), nullptr, s);
  return hipGetLastError() == hipSuccess ? PMR_OK : PMR_E_HIP;
}

int pmr_fft_set_tile(int n, int pass, int columns, int threads, int staging) {
  return set_fft_tile(n, pass, columns, threads, staging) == 0 ? PMR_OK : PMR_E_INVALID;
}

int pmr_paint_set_rows(int n, int channels, int rows) {
  return set_paint_rows(n, channels, rows) == 0 ? PMR_OK : PMR_E_INVALID;
}

int pmr_paint_get_rows(int n, int channels, int* rows) {
  if (!rows || !pow2_in(n, 16, 512) || (channels != 1 && channels != 3)) return PMR_E_INVALID;
  *rows = get_paint_rows(n, channels);
  return PMR_OK;
}

int pmr_fft_set_slab(int n, int columns) {
  return set_fft_slab(n, columns) == 0 ? PMR_OK : PMR_E_INVALID;
}

int pmr_fft_get_slab(int n, int* columns) {
  if (!columns || !pow2_in(n, 16, 512)) return PMR_E_INVALID;
  *columns = get_fft_slab(n);
  return PMR_OK;
}

int pmr_fft_get_tile(int n, int pass, int* columns, int* threads, int* staging) {
  if (!columns || !threads || !staging || !pow2_in(n, 16, 512) || pass < 0 || pass > 2)
    return PMR_E_INVALID;
  get_fft_tile(n, pass, columns, threads, staging);
  return PMR_OK;
}

size_t pmr_sort_scratch_bytes(int n_total, int n_mesh, int batch) {
  if (n_total < 1 || !pow2_in(n_mesh, 16, 512) || batch < 1) return 0;
  return align256((size_t)n_total * sizeof(uint32_t)) +
         cell_sort_scratch_bytes(n_total, (size_t)batch * n_mesh * n_mesh, ilog2((size_t)n_mesh));
}

int pmr_cic_sort(int n_part, int n_mesh, int batch, double box, const double* x,
                 uint32_t* keys_sorted, uint32_t* ids_sorted, uint32_t* row_start, void* scratch,
                 size_t scratch_bytes, void* stream) {
  if (!x || !keys_sorted || !ids_sorted || !row_start || !scratch || !(box > 0) || batch < 1)
    return PMR_E_INVALID;
  if (!pow2_in(n_part, 16, 512) || !pow2_in(n_mesh, 16, 512)) return PMR_E_SHAPE;
  const size_t np3 = (size_t)n_part * n_part * n_part;
  if ((double)batch * np3 >= 2147483648.0 ||
      (double)batch * n_mesh * n_mesh * n_mesh > 4294967296.0)
    return PMR_E_SHAPE;
  const int total = (int)(batch * np3);
  if (scratch_bytes < pmr_sort_scratch_bytes(total, n_mesh, batch)) return PMR_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  uint32_t* keys = (uint32_t*)scratch;
  void* rest = (char*)scratch + align256((size_t)total * sizeof(uint32_t));
  launch_keys(x, ilog2(np3), total, (double)n_mesh / box, n_mesh, keys, nullptr, s);
  launch_cell_sort(keys, nullptr, total, ilog2((size_t)n_mesh), (size_t)batch * n_mesh * n_mesh,
                   keys_sorted, ids_sorted, row_start, rest, nullptr, nullptr, nullptr, s);
  return hipGetLastError() == hipSuccess ? PMR_OK : PMR_E_HIP;
}

int pmr_cic_paint(int n_part, int n_mesh, int batch, double box, const double* x,
                  const uint32_t* keys_sorted, const uint32_t* ids_sorted,
                  const uint32_t* row_start, float mass, float bias, float* out, void* scratch,
                  size_t scratch_bytes, void* stream) {
  if (!x || !keys_sorted || !ids_sorted || !row_start || !out || !scratch || !(box > 0) ||
      batch < 1)
    return PMR_E_INVALID;
  if (!pow2_in(n_part, 16, 512) || !pow2_in(n_mesh, 16, 512)) return PMR_E_SHAPE;
  const size_t np3 = (size_t)n_part * n_part * n_part;
  if ((double)batch * np3 >= 2147483648.0 ||
      (double)batch * n_mesh * n_mesh * n_mesh > 4294967296.0)
    return PMR_E_SHAPE;
  const int total = (int)(batch * np3);
  if (scratch_bytes < (size_t)total * sizeof(Vec3)) return PMR_E_WORKSPACE;
  hipStream_t s = (hipStream_t)stream;
  Vec3* frac = (Vec3*)scratch;
  launch_stream_frac(ids_sorted, x, total, ilog2(np3), n_mesh, box, frac, s);
  launch_paint_mass(keys_sorted, frac, row_start, batch, n_mesh, mass, bias, out, s);
  return hipGetLastError() == hipSuccess ? PMR_OK : PMR_E_HIP;
}

}  // extern "C"
