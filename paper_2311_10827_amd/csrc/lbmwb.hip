// C ABI of liblbmwb (declared in include/lbmwb.h): parameter validation,
// memory layout and kernel launches for the well-balanced phase-field LBM
// step of Ju et al. (arXiv 2311.10827).  The kernels are in forward.h (the
// step) and adjoint.h (its adjoint).
//
// State layout in HBM (planes of the storage type T, each 256-byte aligned):
//   [pop buffer 0][pop buffer 1][S][dphi][mu]
// with NB = 18 (FP64) or 19 (FP32) planes per pop buffer (see common.h).
// A pop buffer holds the post-collision values of the previous step; the
// current pre-collision populations are their pull gather.  Each step reads
// one buffer and writes the other.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "adjoint.h"
#include "forward.h"
#include "step2.h"
#include "lbmwb.h"

using namespace lbm;

// Scratch memory of lbm_step_noalloc, one copy per GPU for the life of the
// process: the step's diagnostic partials, the first-level reduction and the
// reduced diagnostics.  Host code never uses this name as an address (it is a
// host-side stand-in there); the device address comes from
// hipGetSymbolAddress, once per device, at lbm_init (scratch_on_device).
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)4 << 20;
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_BYTES / sizeof(double)];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
bool g_scratch_tried[MAX_DEVICES];
void* g_scratch_ptr[MAX_DEVICES];
hipError_t g_scratch_err[MAX_DEVICES];

// The device address of `scratch` on device `dev` (current when called the
// first time for it), or NULL with *err set if the lookup failed.
void* scratch_on_device(int dev, hipError_t* err) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (dev < 0 || dev >= MAX_DEVICES) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  if (!g_scratch_tried[dev]) {
    void* ptr = nullptr;
    g_scratch_err[dev] = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    g_scratch_ptr[dev] = g_scratch_err[dev] == hipSuccess ? ptr : nullptr;
    g_scratch_tried[dev] = true;
  }
  *err = g_scratch_err[dev];
  return g_scratch_ptr[dev];
}
}  // namespace

// ====================================================================== host
struct lbm_ctx {
  lbm_params p;
  lbm_derived d;
  KP kp;
  int prec;
  size_t esz;
  char* state;
  char* ws;
  hipStream_t stream;
  int cur;
  int scur;             // which of the two S planes holds S_prev
  int64_t step;
  int ntx1, nty1, ntx2, nty2;
  int ntxf, ntyf, hf;   // strips of the fused step kernel and their height
  bool fused_nt;        // the fused step stores streaming (state above the cache size)
  bool fused_xcd;       // the fused step deals its strips to XCDs in contiguous bands
  bool lo16;            // FP32: the low word of f_0 in 16 bits (state above LO16_STATE_BYTES)
  int ntxm, ntym;       // tiles of ka_mu_phi (no more than the K2 tiles, whose
                        // count sizes the parameter partials)
  bool fused;           // lbm_step runs the fused kernel
  bool two_step;        // lbm_step runs pairs of steps as one k_step2 launch
  int w2s, ntx2s, nty2s, h2s; // strips of k_step2: width, counts, height
  bool s2_xcd;          // k_step2 deals its strips to XCDs in contiguous bands
  double* partials;
  double* red_mid;      // [RED_BLOCKS][NQ]: first-level reduction results
  double* diag_dev;     // [2][NQ]: fused step diagnostics, moments diagnostics; then
                        // max |div u| and the five sums of the Laplace jump
  double* diag_host;    // pinned [2][NQ] + 6
  int64_t diag_step;
  bool diag_pending, diag_seen, nonfinite;
  hipEvent_t diag_ev;
  bool timing;
  std::vector<hipEvent_t> tev;  // two events per timed launch
  std::vector<int> tev_steps;   // steps each timed launch advanced
  std::string err;
  bool u0_zero;         // lbm_init got no initial velocity
  int device;           // the GPU current at lbm_init
  double* scratch_dev;  // that GPU's copy of `scratch` (lbm_step_noalloc), or NULL
  hipError_t scratch_err;
  // adjoint workspace (lbm_adjoint_attach)
  char* adj;
  double* th_part;      // [tiles][NTH] parameter-gradient partials
  double* th_out;       // [NTH]
};

namespace {

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int validate(const lbm_params* p, lbm_derived* d) {
  if (!p) return LBM_EINVAL;
  if (p->nx < 1 || p->ny < 1) return LBM_EINVAL;
  if (p->bc_x < 0 || p->bc_x > 1 || p->bc_y < 0 || p->bc_y > 1) return LBM_EINVAL;
  if (p->precision != 32 && p->precision != 64) return LBM_EINVAL;
  if (p->diag_every < 0) return LBM_EINVAL;
  if (p->kernel_path < 0 || p->kernel_path > 3) return LBM_EINVAL;
  // two steps per launch: FP32 on grids periodic in both directions
  if (p->kernel_path == 3 && (p->precision != 32 || p->bc_x != 0 || p->bc_y != 0)) return LBM_EINVAL;
  if (p->nu_form < LBM_NU_LINEAR || p->nu_form > LBM_NU_EXP) return LBM_EINVAL;
  if (p->collision != LBM_BGK && p->collision != LBM_MRT) return LBM_EINVAL;
  if (p->collision == LBM_MRT) {
    for (double r : {p->mrt_f[0], p->mrt_f[1], p->mrt_f[2], p->mrt_f[3], p->mrt_g[0], p->mrt_g[1]})
      if (!(r > 0.0 && r < 2.0)) return LBM_EINVAL;
  }
  const size_t pitch = round_up((size_t)p->nx, 64);
  if (pitch * (size_t)p->ny > (size_t)INT32_MAX) return LBM_EINVAL;
  const double dphi = p->phi_A - p->phi_B;
  if (!(dphi != 0.0) || !std::isfinite(dphi)) return LBM_EINVAL;
  if (p->lo_format < LBM_LO_AUTO || p->lo_format > LBM_LO_32) return LBM_EINVAL;
  if (p->use_tau != 0 && p->use_tau != 1) return LBM_EINVAL;
  // the relaxation parameters: given (alpha, nu_A, nu_B), or derived from
  // the given relaxation times by eq. mobility and the viscosity relation of
  // Sec. 2.3.2, solved for alpha and nu
  double alpha = p->alpha, nuA = p->nu_A, nuB = p->nu_B;
  if (p->use_tau) {
    if (!(p->tau_f > 0.5) || !(p->tau_gA > 0.5) || !(p->tau_gB > 0.5) || !std::isfinite(p->tau_f) ||
        !std::isfinite(p->tau_gA) || !std::isfinite(p->tau_gB))
      return LBM_EINVAL;
    alpha = p->M * INV_CS2 / (p->tau_f - 0.5);
    nuA = CS2 * (p->tau_gA - 0.5);
    nuB = CS2 * (p->tau_gB - 0.5);
  }
  if (!(p->rho_A > 0) || !(p->rho_B > 0) || !(nuA > 0) || !(nuB > 0)) return LBM_EINVAL;
  if (!(p->M > 0) || !(alpha > 0)) return LBM_EINVAL;
  if (!std::isfinite(p->rho_A) || !std::isfinite(p->rho_B) || !std::isfinite(nuA) ||
      !std::isfinite(nuB) || !std::isfinite(p->M) || !std::isfinite(alpha))
    return LBM_EINVAL;
  if (!std::isfinite(p->gx) || !std::isfinite(p->gy)) return LBM_EINVAL;
  double kappa = p->kappa, beta = p->beta;
  if (p->use_sigma_W) {
    if (!(p->sigma > 0) || !(p->W > 0)) return LBM_EINVAL;
    // eq. beta and eq. suiface_tension solved for kappa and beta
    kappa = 1.5 * p->sigma * p->W / (dphi * dphi);
    beta = 8.0 * kappa / (p->W * p->W * dphi * dphi);
  }
  if (!(kappa >= 0) || !(beta >= 0) || !std::isfinite(kappa) || !std::isfinite(beta))
    return LBM_EINVAL;
  lbm_derived r;
  r.kappa = kappa;
  r.beta = beta;
  const double ad = std::fabs(dphi);
  r.sigma = ad * ad * ad * std::sqrt(2.0 * kappa * beta) / 6.0;
  r.W = beta > 0 ? std::sqrt(8.0 * kappa / (beta * dphi * dphi)) : 0.0;
  r.alpha = alpha;
  r.nu_A = nuA;
  r.nu_B = nuB;
  if (p->use_tau) {
    r.tau_f = p->tau_f;
    r.tau_gA = p->tau_gA;
    r.tau_gB = p->tau_gB;
  } else {
    // eq. mobility and the viscosity relation of Sec. 2.3.2, solved for tau
    r.tau_f = 0.5 + p->M * INV_CS2 / alpha;
    r.tau_gA = 0.5 + nuA * INV_CS2;
    r.tau_gB = 0.5 + nuB * INV_CS2;
  }
  if (!(r.tau_f > 0.5) || !(r.tau_gA > 0.5) || !(r.tau_gB > 0.5)) return LBM_EINVAL;
  r.lo16 = 0;
  r.two_step = 0;
  if (d) *d = r;
  return LBM_OK;
}

struct Layout {
  size_t pitch, ps, esz, nb;
  size_t state_bytes, ws_bytes;
  int ntx1, nty1, ntx2, nty2;
  int ntxf, ntyf;       // strips of the fused step kernel
  bool fused;           // lbm_step runs the fused kernel
};

constexpr int ADJ_PLANES = 7;
// fused step launches aim at no fewer workgroups than this (8 per CU)
constexpr long long FUSED_MIN_BLOCKS = 2048;
// kernel_path 0 runs the fused step when the grid gives at least this many
// strips of 256 x 8 cells
constexpr long long FUSED_AUTO_STRIPS_32 = 512, FUSED_AUTO_STRIPS_64 = 512;
// above this state size the fused step stores streaming (MI355X has a 256 MB
// last-level cache; a state that fits is read back from it)
constexpr size_t FUSED_CACHED_STATE_BYTES = (size_t)224 << 20;
// FP32 fused launches of at least this many workgroups take their strips in
// dispatch order (consecutive strips of a band on different XCDs) instead of
// in XCD-contiguous bands: measured on MI355X, 1-2 % faster at 8192^2 and
// 16384^2 in FP32 (over three allocations at 16384^2), but 6 % slower at
// 4096^2 and 3 % at 1024^2 in FP32, and 1.5-3 % slower at 16384^2 in FP64
constexpr long long FUSED_DISPATCH_ORDER_BLOCKS_32 = 8192;
// k_step2 launches aim at no fewer workgroups than this (two rounds of two
// per CU): at 4096^2 on MI355X, 128-row strips (608 workgroups) were a fifth
// slower than 64-row ones; at 16384^2 the 128-row strips are 3 % faster than
// 64-row ones
constexpr long long S2_MIN_BLOCKS = 1024;
// k_step2: resident workgroups per CU (its 175 VGPRs and 74 KB of LDS), and
// the lowest strip height the round-filling choice considers
constexpr int S2_WG_PER_CU = 2;
constexpr int S2_ROUND_H_MIN = 48;
// FP32 fused step: resident workgroups per CU (its 48 KB of LDS), and the
// range of strip heights and the launch size (in rounds of resident
// workgroups) within which the height is chosen to fill the last round
constexpr int FUSED32_WG_PER_CU = 3;
constexpr int FUSED_ROUND_H_MIN = 24, FUSED_ROUND_H_MAX = 48;
constexpr long long FUSED_FEW_ROUNDS = 4;
// above this FP32 state size the low word of f_0 is kept in 16 bits: 2 % off
// the HBM-bound step from 4096^2 up, 3 % on at 2048^2 where its arithmetic
// is not hidden
constexpr size_t LO16_STATE_BYTES = (size_t)1 << 30;

bool two_step_of(const lbm_params* p, size_t state_bytes);

// FP32: the low word of f_0 in 16 bits (lbm_params.lo_format; automatic:
// for states above LO16_STATE_BYTES that the one-step kernels run, where
// the step is bound by HBM and the 16-bit word pays; the two-step kernel is
// bound by instruction latency instead, and keeps the 32-bit word: 16384^2
// on MI355X, 5.00 against 5.45 ms per step)
bool lo16_of(const lbm_params* p, size_t state_bytes) {
  if (p->precision != 32) return false;
  if (p->lo_format == LBM_LO_16) return true;
  if (p->lo_format == LBM_LO_32) return false;
  return state_bytes > LO16_STATE_BYTES && !two_step_of(p, state_bytes);
}

// Two steps per launch (k_step2): asked for (kernel_path 3), or automatic
// for FP32 states on periodic grids beyond the last-level cache (measured on
// MI355X, against the fused single step: 16384^2 4.60 against 7.49 ms per
// step, 4096^2 0.31 against 0.53, 2048^2 0.114 against 0.15; at 1024^2,
// where the single step runs from the cache, 0.040 against 0.036 ms)
bool two_step_of(const lbm_params* p, size_t state_bytes) {
  if (p->kernel_path == 3) return true;
  return p->kernel_path == 0 && p->precision == 32 && p->bc_x == 0 && p->bc_y == 0 &&
         state_bytes > FUSED_CACHED_STATE_BYTES;
}

// Parameter-gradient partials: one slot per K2 tile of ka_local (ka_mu_phi
// has no more tiles than that).
size_t th_tiles(const lbm_params* p) {
  return (size_t)((p->nx + K2_TX - 1) / K2_TX) * ((p->ny + K2_TY - 1) / K2_TY);
}

size_t adj_plane_bytes(const lbm_params* p) {
  return round_up((size_t)p->nx * p->ny * (p->precision == 32 ? 4 : 8), 256);
}

size_t adj_bytes(const lbm_params* p) {
  return ADJ_PLANES * adj_plane_bytes(p) + round_up((th_tiles(p) + 1) * NTH * sizeof(double), 256);
}

Layout layout_of(const lbm_params* p) {
  Layout L;
  L.esz = p->precision == 32 ? 4 : 8;
  L.nb = p->precision == 32 ? Store<float>::NB : Store<double>::NB;
  L.pitch = round_up((size_t)p->nx, 64);
  // Plane stride: 256-byte multiple plus 4 KiB of padding so that the 18
  // planes read together do not sit at addresses a power of two apart.
  L.ps = round_up(L.pitch * (size_t)p->ny, 256 / L.esz) + 4096 / L.esz;
  // two population buffers, two S planes (k_step2 reads one and writes the
  // other), the phi and mu planes
  L.state_bytes = (2 * L.nb + 4) * L.ps * L.esz;
  L.ntx1 = (p->nx + K1_TX - 1) / K1_TX;
  L.nty1 = (p->ny + K1_TY - 1) / K1_TY;
  L.ntx2 = (p->nx + K2_TX - 1) / K2_TX;
  L.nty2 = (p->ny + K2_TY - 1) / K2_TY;
  const size_t nparts = (size_t)L.ntx2 * L.nty2;
  // partials, first-level reduction, [2][NQ] diagnostics, max |div u| and
  // the five sums of the Laplace jump
  L.ws_bytes = round_up((nparts * NQ + (RED_BLOCKS + 2) * NQ + 6) * sizeof(double), 256);
  return L;
}

#define HIPCHK(ctx, expr)                                                  \
  do {                                                                     \
    hipError_t e_ = (expr);                                                \
    if (e_ != hipSuccess) {                                                \
      (ctx)->err = std::string(#expr) + ": " + hipGetErrorString(e_);     \
      return LBM_EHIP;                                                     \
    }                                                                      \
  } while (0)

#define LAUNCHCHK(ctx) HIPCHK(ctx, hipGetLastError())

template <typename T>
T* plane(lbm_ctx* c, int k) {
  return reinterpret_cast<T*>(c->state) + (size_t)k * c->kp.ps;
}
template <typename T>
T* popbuf(lbm_ctx* c, int which) {
  return plane<T>(c, which * Store<T>::NB);
}
template <typename T>
T* S_plane(lbm_ctx* c) { return plane<T>(c, 2 * Store<T>::NB + c->scur); }
template <typename T>
T* S_alt(lbm_ctx* c) { return plane<T>(c, 2 * Store<T>::NB + (c->scur ^ 1)); }
template <typename T>
T* dphi_plane(lbm_ctx* c) { return plane<T>(c, 2 * Store<T>::NB + 2); }
template <typename T>
T* mu_plane(lbm_ctx* c) { return plane<T>(c, 2 * Store<T>::NB + 3); }

unsigned blocks_for(long long n) { return (unsigned)((n + 255) / 256); }

// The kernels that read or write the FP32 low word of f_0 take its format as
// a template argument (LO16); f is called with std::true_type for an FP32
// context that keeps it in 16 bits, else with std::false_type.
template <typename T, typename F>
void lo_dispatch(const lbm_ctx* c, F&& f) {
  if (std::is_same<T, float>::value && c->lo16)
    f(std::true_type{});
  else
    f(std::false_type{});
}

// A "state" is a pop buffer (NB planes) plus an S_prev plane.  The context's
// own state is its current pop buffer with the shared S plane; a snapshot
// holds NB + 1 consecutive planes in the same layout.
template <typename T>
void launch_phi_mu_k(lbm_ctx* c, const T* B, T* dphi, T* mu) {
  lo_dispatch<T>(c, [&](auto lo) {
    constexpr bool L16 = decltype(lo)::value && std::is_same<T, float>::value;
    hipLaunchKernelGGL((k_phi_mu<T, false, L16>), dim3(c->ntx1 * c->nty1), dim3(256), 0, c->stream, c->kp,
                       B, nullptr, dphi, mu, c->ntx1);
  });
}
template <typename T>
int launch_phi_mu(lbm_ctx* c, const T* B) {
  launch_phi_mu_k<T>(c, B, dphi_plane<T>(c), mu_plane<T>(c));
  LAUNCHCHK(c);
  return LBM_OK;
}
template <typename T>
int launch_phi_mu(lbm_ctx* c) {
  return launch_phi_mu<T>(c, popbuf<T>(c, c->cur));
}

// The collide-stream pass; the MRT instantiation for the modes that collide.
template <typename T, int MODE>
int launch_collide(lbm_ctx* c, MomOut mo, const T* Bin, T* Bout, const T* Sin, T* Sout, const T* dphi,
                   const T* mu) {
  constexpr bool COLLIDES = MODE == M_STEP || MODE == M_STEP_DIAG;
  lo_dispatch<T>(c, [&](auto lo) {
    constexpr bool L16 = decltype(lo)::value && std::is_same<T, float>::value;
    if (COLLIDES && c->kp.collision == LBM_MRT)
      hipLaunchKernelGGL((k_collide<T, MODE, COLLIDES, L16>), dim3(c->ntx2 * c->nty2), dim3(256), 0,
                         c->stream, c->kp, Bin, Bout, Sin, Sout, dphi, mu, mo, c->partials, c->ntx2);
    else
      hipLaunchKernelGGL((k_collide<T, MODE, false, L16>), dim3(c->ntx2 * c->nty2), dim3(256), 0, c->stream,
                         c->kp, Bin, Bout, Sin, Sout, dphi, mu, mo, c->partials, c->ntx2);
  });
  LAUNCHCHK(c);
  return LBM_OK;
}
template <typename T, int MODE>
int launch_collide(lbm_ctx* c, MomOut mo, const T* Bin, T* Bout, const T* Sin, T* Sout) {
  return launch_collide<T, MODE>(c, mo, Bin, Bout, Sin, Sout, dphi_plane<T>(c), mu_plane<T>(c));
}
template <typename T, int MODE>
int launch_collide(lbm_ctx* c, MomOut mo) {
  return launch_collide<T, MODE>(c, mo, popbuf<T>(c, c->cur), popbuf<T>(c, c->cur ^ 1), S_plane<T>(c),
                                 S_plane<T>(c));
}

template <typename T, int MODE, bool WRITE_PHIMU, bool MRT, bool NT>
void launch_fused_k(lbm_ctx* c, const T* Bin, T* Bout, const T* Sin, T* Sout, T* dphi, T* mu) {
  lo_dispatch<T>(c, [&](auto lo) {
    constexpr bool L16 = decltype(lo)::value && std::is_same<T, float>::value;
    hipLaunchKernelGGL((k_step_fused<T, MODE, WRITE_PHIMU, MRT, NT, L16>), dim3(c->ntxf * c->ntyf),
                       dim3(Strip<T>::W), 0, c->stream, c->kp, Bin, Bout, Sin, Sout, dphi, mu, c->partials,
                       c->ntxf, c->hf, c->fused_xcd ? 1 : 0);
  });
}
template <typename T, int MODE, bool WRITE_PHIMU>
int launch_fused(lbm_ctx* c, const T* Bin, T* Bout, const T* Sin, T* Sout, T* dphi, T* mu) {
  const bool mrt = c->kp.collision == LBM_MRT;
  if (c->fused_nt) {
    if (mrt)
      launch_fused_k<T, MODE, WRITE_PHIMU, true, true>(c, Bin, Bout, Sin, Sout, dphi, mu);
    else
      launch_fused_k<T, MODE, WRITE_PHIMU, false, true>(c, Bin, Bout, Sin, Sout, dphi, mu);
  } else {
    if (mrt)
      launch_fused_k<T, MODE, WRITE_PHIMU, true, false>(c, Bin, Bout, Sin, Sout, dphi, mu);
    else
      launch_fused_k<T, MODE, WRITE_PHIMU, false, false>(c, Bin, Bout, Sin, Sout, dphi, mu);
  }
  LAUNCHCHK(c);
  return LBM_OK;
}

// Diagnostic partials one step writes: one per strip of the fused kernels,
// one per tile of the collide pass.
long long step_partials(const lbm_ctx* c) {
  if (c->fused) return (long long)c->ntxf * c->ntyf;
  return (long long)c->ntx2 * c->nty2;
}

int launch_reduce(lbm_ctx* c, int slot, long long n) {
  const long long chunk = (n + RED_BLOCKS - 1) / RED_BLOCKS;
  const long long nb = (n + chunk - 1) / chunk;
  hipLaunchKernelGGL(k_reduce_diag, dim3((unsigned)nb), dim3(256), 0, c->stream, c->partials, n, chunk,
                     c->red_mid);
  LAUNCHCHK(c);
  hipLaunchKernelGGL(k_reduce_diag, dim3(1), dim3(256), 0, c->stream, c->red_mid, nb, nb,
                     c->diag_dev + slot * NQ);
  LAUNCHCHK(c);
  return LBM_OK;
}

// v: the NQ reduced quantities; x: max |div u| and the five sums of the
// Laplace jump (lbm_moments), or NULL for the fused step's diagnostics,
// which form neither (max_div_u = -1, no bulk cells).
void fill_diag(const double* v, int64_t step, lbm_diag* d, const double* x) {
  d->sum_phi = v[0];
  d->source_sum = v[1];
  d->kinetic_energy = v[2];
  d->max_u = v[3];
  d->min_rho = v[4];
  d->max_rho = v[5];
  d->mu_min = v[6];
  d->mu_max = v[7];
  d->phi_min = v[8];
  d->phi_max = v[9];
  d->max_div_u = x ? x[0] : -1.0;
  d->n_bulk_A = x ? (int64_t)x[2] : 0;
  d->n_bulk_B = x ? (int64_t)x[4] : 0;
  // both bulk sets non-empty and disjoint (an interface between them)
  d->laplace_dP = x && x[2] > 0 && x[4] > 0 && x[5] == 0 ? x[1] / x[2] - x[3] / x[4] : 0.0;
  d->n_nonfinite = (int64_t)v[10];
  d->step = step;
}

bool diag_bad(const double* v) { return v[10] > 0 || !(v[4] > 0); }

// Consume a completed fused-diagnostic result; `wait` blocks until it is.
int consume_diag(lbm_ctx* c, bool wait) {
  if (!c->diag_pending) return LBM_OK;
  if (wait) {
    HIPCHK(c, hipEventSynchronize(c->diag_ev));
  } else {
    hipError_t q = hipEventQuery(c->diag_ev);
    if (q == hipErrorNotReady) return LBM_OK;
    if (q != hipSuccess) {
      c->err = std::string("hipEventQuery: ") + hipGetErrorString(q);
      return LBM_EHIP;
    }
  }
  c->diag_pending = false;
  c->diag_seen = true;
  if (diag_bad(c->diag_host)) c->nonfinite = true;
  return LBM_OK;
}

// One step: the fused kernel (phi and mu stay in LDS), or the phi/mu pass
// then the collide-stream pass.
template <typename T>
int launch_step(lbm_ctx* c, bool diag) {
  if (c->fused) {
    T* Bin = popbuf<T>(c, c->cur);
    T* Bout = popbuf<T>(c, c->cur ^ 1);
    return diag ? launch_fused<T, M_STEP_DIAG, false>(c, Bin, Bout, S_plane<T>(c), S_plane<T>(c), nullptr, nullptr)
                : launch_fused<T, M_STEP, false>(c, Bin, Bout, S_plane<T>(c), S_plane<T>(c), nullptr, nullptr);
  }
  int r = launch_phi_mu<T>(c);
  if (r) return r;
  return diag ? launch_collide<T, M_STEP_DIAG>(c, MomOut{}) : launch_collide<T, M_STEP>(c, MomOut{});
}

// Two steps as one k_step2 launch (FP32, periodic): the state advances by
// two steps and S moves to the other S plane.
template <bool MRT, bool NT>
void launch_step2_k(lbm_ctx* c, const float* Bin, float* Bout, const float* Sin, float* Sout) {
  lo_dispatch<float>(c, [&](auto lo) {
    constexpr bool L16 = decltype(lo)::value;
    hipLaunchKernelGGL((k_step2<MRT, NT, L16>), dim3(c->ntx2s * c->nty2s), dim3(S2_L), 0, c->stream, c->kp,
                       Bin, Bout, Sin, Sout, c->w2s, c->ntx2s, c->h2s, c->s2_xcd ? 1 : 0);
  });
}
int launch_step2(lbm_ctx* c) {
  const float* Bin = popbuf<float>(c, c->cur);
  float* Bout = popbuf<float>(c, c->cur ^ 1);
  const float* Sin = S_plane<float>(c);
  float* Sout = S_alt<float>(c);
  const bool mrt = c->kp.collision == LBM_MRT;
  if (c->fused_nt) {
    if (mrt)
      launch_step2_k<true, true>(c, Bin, Bout, Sin, Sout);
    else
      launch_step2_k<false, true>(c, Bin, Bout, Sin, Sout);
  } else {
    if (mrt)
      launch_step2_k<true, false>(c, Bin, Bout, Sin, Sout);
    else
      launch_step2_k<false, false>(c, Bin, Bout, Sin, Sout);
  }
  LAUNCHCHK(c);
  return LBM_OK;
}

template <typename T>
int step_impl(lbm_ctx* c, int64_t n) {
  for (int64_t k = 0; k < n; ++k) {
    const bool diag = c->p.diag_every > 0 && (c->step % c->p.diag_every) == 0;
    // two steps in one launch when neither is due for diagnostics
    const bool pair = std::is_same<T, float>::value && c->two_step && k + 1 < n && !diag &&
                      !(c->p.diag_every > 0 && ((c->step + 1) % c->p.diag_every) == 0);
    auto launch = [&]() { return pair ? launch_step2(c) : launch_step<T>(c, diag); };
    if (c->timing) {
      hipEvent_t e[2];
      for (int j = 0; j < 2; ++j) {
        HIPCHK(c, hipEventCreate(&e[j]));
        c->tev.push_back(e[j]);
      }
      c->tev_steps.push_back(pair ? 2 : 1);
      HIPCHK(c, hipEventRecord(e[0], c->stream));
      int r = launch();
      if (r) return r;
      HIPCHK(c, hipEventRecord(e[1], c->stream));
    } else {
      int r = launch();
      if (r) return r;
    }
    if (pair) {
      c->cur ^= 1;
      c->scur ^= 1;
      c->step += 2;
      k += 1;
      continue;
    }
    if (diag) {
      int r = consume_diag(c, true);  // the host buffer is about to be reused
      if (r) return r;
      r = launch_reduce(c, 0, step_partials(c));
      if (r) return r;
      HIPCHK(c, hipMemcpyAsync(c->diag_host, c->diag_dev, NQ * sizeof(double),
                               hipMemcpyDeviceToHost, c->stream));
      HIPCHK(c, hipEventRecord(c->diag_ev, c->stream));
      c->diag_pending = true;
      c->diag_step = c->step;
    }
    c->cur ^= 1;
    c->step += 1;
  }
  return LBM_OK;
}

template <typename T>
int init_impl(lbm_ctx* c, const double* phi0, const double* ux0, const double* uy0) {
  hipLaunchKernelGGL((k_phi_mu<T, true>), dim3(c->ntx1 * c->nty1), dim3(256), 0, c->stream, c->kp,
                     nullptr, phi0, dphi_plane<T>(c), mu_plane<T>(c), c->ntx1);
  LAUNCHCHK(c);
  const long long n = (long long)c->p.nx * c->p.ny;
  lo_dispatch<T>(c, [&](auto lo) {
    constexpr bool L16 = decltype(lo)::value && std::is_same<T, float>::value;
    hipLaunchKernelGGL((k_init_pops<T, L16>), dim3(blocks_for(n)), dim3(256), 0, c->stream, c->kp,
                       popbuf<T>(c, c->cur), phi0, ux0, uy0, mu_plane<T>(c));
  });
  LAUNCHCHK(c);
  int r = launch_phi_mu<T>(c);
  if (r) return r;
  return launch_collide<T, M_INIT_S>(c, MomOut{});
}

template <typename T>
int moments_impl(lbm_ctx* c, MomOut mo, lbm_diag* diag) {
  int r = launch_phi_mu<T>(c);
  if (r) return r;
  // max |div u| and the Laplace jump need u, phi, mu and p of every cell.
  // Where the caller asks for diagnostics without those planes, the moments
  // kernel writes them into the population buffer the next step overwrites
  // entirely (it holds 18 or 19 planes; five dense FP64 planes fit).
  const long long n = (long long)c->p.nx * c->p.ny;
  if (diag) {
    double* scratch = reinterpret_cast<double*>(popbuf<T>(c, c->cur ^ 1));
    if (!mo.ux) mo.ux = scratch;
    if (!mo.uy) mo.uy = scratch + n;
    if (!mo.phi) mo.phi = scratch + 2 * n;
    if (!mo.mu) mo.mu = scratch + 3 * n;
    if (!mo.p) mo.p = scratch + 4 * n;
  }
  r = launch_collide<T, M_MOMENTS>(c, mo);
  if (r) return r;
  if (diag) {
    r = launch_reduce(c, 1, (long long)c->ntx2 * c->nty2);
    if (r) return r;
    // the first-level reduction area is free again: it takes the partials
    hipLaunchKernelGGL(k_max_div_u, dim3(RED_BLOCKS), dim3(256), 0, c->stream, c->kp, mo.ux, mo.uy,
                       c->red_mid);
    LAUNCHCHK(c);
    hipLaunchKernelGGL(k_max_reduce, dim3(1), dim3(256), 0, c->stream, c->red_mid, RED_BLOCKS,
                       c->diag_dev + 2 * NQ);
    LAUNCHCHK(c);
    // the phi extrema of the moments diagnostics set the bulk thresholds
    hipLaunchKernelGGL(k_laplace_part, dim3(RED_BLOCKS), dim3(256), 0, c->stream, c->kp, mo.phi, mo.mu,
                       mo.p, c->diag_dev + NQ + 8, c->red_mid);
    LAUNCHCHK(c);
    hipLaunchKernelGGL(k_laplace_reduce, dim3(1), dim3(256), 0, c->stream, c->red_mid, RED_BLOCKS,
                       c->diag_dev + 2 * NQ + 1);
    LAUNCHCHK(c);
    HIPCHK(c, hipMemcpyAsync(c->diag_host + NQ, c->diag_dev + NQ, (NQ + 6) * sizeof(double),
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    fill_diag(c->diag_host + NQ, c->step, diag, c->diag_host + 2 * NQ);
  }
  return LBM_OK;
}

template <typename T>
int get_state_impl(lbm_ctx* c, int x0, int y0, int w, int h, double* f, double* g, double* Sp) {
  const long long n = (long long)w * h;
  lo_dispatch<T>(c, [&](auto lo) {
    constexpr bool L16 = decltype(lo)::value && std::is_same<T, float>::value;
    hipLaunchKernelGGL((k_get_state<T, L16>), dim3(blocks_for(n)), dim3(256), 0, c->stream, c->kp,
                       popbuf<T>(c, c->cur), S_plane<T>(c), x0, y0, w, h, f, g, Sp);
  });
  LAUNCHCHK(c);
  return LBM_OK;
}

template <typename T>
int set_state_impl(lbm_ctx* c, const double* f, const double* g, const double* Sp) {
  const long long n = (long long)c->p.nx * c->p.ny;
  lo_dispatch<T>(c, [&](auto lo) {
    constexpr bool L16 = decltype(lo)::value && std::is_same<T, float>::value;
    hipLaunchKernelGGL((k_set_state<T, L16>), dim3(blocks_for(n)), dim3(256), 0, c->stream, c->kp,
                       popbuf<T>(c, c->cur), S_plane<T>(c), f, g, Sp);
  });
  LAUNCHCHK(c);
  return LBM_OK;
}

template <typename T>
AdjWork<T> adj_work(lbm_ctx* c) {
  const size_t pb = adj_plane_bytes(&c->p);
  T* q[ADJ_PLANES];
  for (int k = 0; k < ADJ_PLANES; ++k) q[k] = reinterpret_cast<T*>(c->adj + k * pb);
  return AdjWork<T>{q[0], q[1], q[2], q[3], q[4], q[5], q[6]};
}

// Snapshot layout: [NB pop planes][S_prev][dphi][mu], plane stride as in the
// state.  The phi/mu planes are scratch that lbm_step_into fills for its
// source, so the adjoint of that state need not recompute them.
template <typename T>
T* snap_S(const lbm_ctx* c, const T* snap) {
  return const_cast<T*>(snap) + (size_t)Store<T>::NB * c->kp.ps;
}
template <typename T>
T* snap_dphi(const lbm_ctx* c, const T* snap) {
  return snap_S(c, snap) + c->kp.ps;
}
template <typename T>
T* snap_mu(const lbm_ctx* c, const T* snap) {
  return snap_S(c, snap) + 2 * c->kp.ps;
}

template <typename T>
int step_into_impl(lbm_ctx* c, T* src, T* dst) {
  if (c->fused)
    return launch_fused<T, M_STEP, true>(c, src, dst, snap_S(c, src), snap_S(c, dst), snap_dphi(c, src),
                                         snap_mu(c, src));
  launch_phi_mu_k<T>(c, src, snap_dphi(c, src), snap_mu(c, src));
  LAUNCHCHK(c);
  return launch_collide<T, M_STEP>(c, MomOut{}, src, dst, snap_S(c, src), snap_S(c, dst),
                                  snap_dphi(c, src), snap_mu(c, src));
}

template <typename T>
int adjoint_step_impl(lbm_ctx* c, T* state, const T* lam_in, T* lam_out, bool have_phi_mu) {
  T* dphi = snap_dphi(c, state);
  T* mu = snap_mu(c, state);
  if (!have_phi_mu) {
    launch_phi_mu_k<T>(c, state, dphi, mu);
    LAUNCHCHK(c);
  }
  const unsigned nb = (unsigned)(c->ntx2 * c->nty2);
  const AdjWork<T> w = adj_work<T>(c);
  // periodic grids: ka_local's wall-free form (scalar row bases)
  const bool per = !c->kp.bcx && !c->kp.bcy;
  if (c->kp.collision == LBM_MRT) {
    if (per)
      hipLaunchKernelGGL((ka_local<T, false, true, true>), dim3(nb), dim3(256), 0, c->stream, c->kp, state, dphi,
                         mu, lam_in, lam_out, w, c->th_part, c->ntx2);
    else
      hipLaunchKernelGGL((ka_local<T, false, true>), dim3(nb), dim3(256), 0, c->stream, c->kp, state, dphi, mu,
                         lam_in, lam_out, w, c->th_part, c->ntx2);
    LAUNCHCHK(c);
    hipLaunchKernelGGL((ka_mu_phi<T, false, true>), dim3(c->ntxm * c->ntym), dim3(KM_THREADS), 0, c->stream,
                       c->kp, dphi, lam_in, lam_out, w, c->th_part, c->ntxm);
  } else {
    if (per)
      hipLaunchKernelGGL((ka_local<T, false, false, true>), dim3(nb), dim3(256), 0, c->stream, c->kp, state,
                         dphi, mu, lam_in, lam_out, w, c->th_part, c->ntx2);
    else
      hipLaunchKernelGGL((ka_local<T, false>), dim3(nb), dim3(256), 0, c->stream, c->kp, state, dphi, mu,
                         lam_in, lam_out, w, c->th_part, c->ntx2);
    LAUNCHCHK(c);
    hipLaunchKernelGGL((ka_mu_phi<T, false>), dim3(c->ntxm * c->ntym), dim3(KM_THREADS), 0, c->stream,
                       c->kp, dphi, lam_in, lam_out, w, c->th_part, c->ntxm);
  }
  LAUNCHCHK(c);
  return LBM_OK;
}

// Recompute the states of one checkpoint segment (snaps[0] holds s_k, the
// others receive s_{k+1}..s_{k+L-1}) and run the L adjoint steps in reverse,
// ping-ponging lambda between lam and tmp.  Returns the buffer holding
// dL/ds_k in *which (0: lam, 1: tmp).
template <typename T>
int adjoint_segment_impl(lbm_ctx* c, T* const* snaps, int L, T* lam, T* tmp, int* which) {
  for (int k = 1; k < L; ++k) {
    int r = step_into_impl<T>(c, snaps[k - 1], snaps[k]);
    if (r) return r;
  }
  T* a = lam;
  T* b = tmp;
  for (int k = L - 1; k >= 0; --k) {
    int r = adjoint_step_impl<T>(c, snaps[k], a, b, k < L - 1);
    if (r) return r;
    T* t = a;
    a = b;
    b = t;
  }
  *which = a == lam ? 0 : 1;
  return LBM_OK;
}

template <typename T>
int adjoint_init_impl(lbm_ctx* c, const T* state, const double* phi0, const T* lam0, T* scratch,
                      double* dphi0) {
  int r = launch_phi_mu<T>(c, state);
  if (r) return r;
  const unsigned nb = (unsigned)(c->ntx2 * c->nty2);
  const AdjWork<T> w = adj_work<T>(c);
  hipLaunchKernelGGL((ka_local<T, true>), dim3(nb), dim3(256), 0, c->stream, c->kp, state, dphi_plane<T>(c),
                     mu_plane<T>(c), lam0, scratch, w, c->th_part, c->ntx2);
  LAUNCHCHK(c);
  hipLaunchKernelGGL((ka_mu_phi<T, true>), dim3(c->ntxm * c->ntym), dim3(KM_THREADS), 0, c->stream, c->kp,
                     dphi_plane<T>(c), lam0, scratch, w, c->th_part, c->ntxm);
  LAUNCHCHK(c);
  // mu0 = mu(phi0) into the mu plane
  hipLaunchKernelGGL((k_phi_mu<T, true>), dim3(c->ntx1 * c->nty1), dim3(256), 0, c->stream, c->kp, nullptr,
                     phi0, dphi_plane<T>(c), mu_plane<T>(c), c->ntx1);
  LAUNCHCHK(c);
  hipLaunchKernelGGL(ki_local<T>, dim3(nb), dim3(256), 0, c->stream, c->kp, phi0, mu_plane<T>(c), lam0,
                     scratch, w, c->th_part, c->ntx2);
  LAUNCHCHK(c);
  hipLaunchKernelGGL(ki_phi<T>, dim3(nb), dim3(256), 0, c->stream, c->kp, phi0, w, dphi0, c->th_part,
                     c->ntx2);
  LAUNCHCHK(c);
  return LBM_OK;
}

size_t snapshot_bytes(const lbm_ctx* c) {
  const size_t nb = c->prec == 64 ? Store<double>::NB : Store<float>::NB;
  return (nb + 3) * (size_t)c->kp.ps * c->esz;
}

}  // namespace

extern "C" {

int lbm_derive(const lbm_params* p, lbm_derived* out) {
  int r = validate(p, out);
  if (r == LBM_OK && out) {
    out->lo16 = lo16_of(p, layout_of(p).state_bytes) ? 1 : 0;
    out->two_step = two_step_of(p, layout_of(p).state_bytes) ? 1 : 0;
  }
  return r;
}

size_t lbm_state_bytes(const lbm_params* p) {
  if (validate(p, nullptr) != LBM_OK) return 0;
  return layout_of(p).state_bytes;
}

size_t lbm_workspace_bytes(const lbm_params* p) {
  if (validate(p, nullptr) != LBM_OK) return 0;
  return layout_of(p).ws_bytes;
}

int lbm_init(lbm_ctx** out, const lbm_params* p, void* state, void* workspace, const double* phi0,
             const double* ux0, const double* uy0, void* stream) {
  if (!out) return LBM_EINVAL;
  *out = nullptr;
  lbm_derived d;
  int r = validate(p, &d);
  if (r) return r;
  if (!state || !workspace || !phi0) return LBM_EINVAL;
  if (((uintptr_t)state & 255) || ((uintptr_t)workspace & 255)) return LBM_EINVAL;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return LBM_EHIP;
  lbm_ctx* c = new lbm_ctx();
  c->p = *p;
  c->d = d;
  c->device = dev;
  // set-up of lbm_step_noalloc's scratch on this device (its failure only
  // disables that entry point, which then reports it)
  c->scratch_dev = static_cast<double*>(scratch_on_device(dev, &c->scratch_err));
  const Layout L = layout_of(p);
  c->prec = p->precision;
  c->esz = L.esz;
  c->state = static_cast<char*>(state);
  c->ws = static_cast<char*>(workspace);
  c->stream = static_cast<hipStream_t>(stream);
  c->cur = 0;
  c->scur = 0;
  c->step = 0;
  c->ntx1 = L.ntx1;
  c->nty1 = L.nty1;
  c->ntx2 = L.ntx2;
  c->nty2 = L.nty2;
  {
    // Strip height: the full height, halved (down to 8 rows; each strip
    // recomputes phi on 4 rows beyond its own) while the launch has fewer
    // than FUSED_MIN_BLOCKS workgroups.
    const int sw = p->precision == 32 ? Strip<float>::W : Strip<double>::W;
    int sh = p->precision == 32 ? Strip<float>::H : Strip<double>::H;
    c->ntxf = (p->nx + sw - 1) / sw;
    while (sh > 8 && (long long)c->ntxf * ((p->ny + sh - 1) / sh) < FUSED_MIN_BLOCKS) sh /= 2;
    c->hf = sh;
    c->ntyf = (p->ny + sh - 1) / sh;
    c->fused_xcd = !(p->precision == 32 && (long long)c->ntxf * c->ntyf >= FUSED_DISPATCH_ORDER_BLOCKS_32);
    // FP32 states beyond the last-level cache whose launch is only a few
    // rounds of resident workgroups: a strip height that makes the strip
    // count a whole number of rounds leaves no part-empty last round, and
    // the strips go in dispatch order (4096^2: 43-row strips, exactly two
    // rounds, 0.539 against 0.555 ms per step with 32-row strips in XCD
    // bands on MI355X)
    int cus = 0;
    if (p->precision == 32 && L.state_bytes > FUSED_CACHED_STATE_BYTES && sh == Strip<float>::H &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0) {
      const long long slots = (long long)FUSED32_WG_PER_CU * cus;
      if ((long long)c->ntxf * c->ntyf < FUSED_FEW_ROUNDS * slots) {
        double best = -1.0;
        for (int h = FUSED_ROUND_H_MIN; h <= FUSED_ROUND_H_MAX; ++h) {
          const long long n = (long long)c->ntxf * ((p->ny + h - 1) / h);
          const double eff = (double)n / (double)(((n + slots - 1) / slots) * slots);
          const bool closer = std::abs(h - Strip<float>::H) < std::abs(c->hf - Strip<float>::H);
          if (eff > best + 1e-9 || (eff > best - 1e-9 && closer)) {
            best = eff;
            c->hf = h;
          }
        }
        c->ntyf = (p->ny + c->hf - 1) / c->hf;
        c->fused_xcd = false;
      }
    }
  }
  c->ntxm = (p->nx + KM_TX - 1) / KM_TX;
  c->ntym = (p->ny + KM_TY - 1) / KM_TY;
  {
    // Automatic choice: the fused kernel marches its strips row by row, so
    // on grids that give it few strips even at the lowest height its serial
    // rows cost more than the second kernel's round trip of phi and mu
    // (measured crossover: between 768^2 and 1024^2 in both precisions).
    const long long strips8 = (long long)c->ntxf * ((p->ny + 7) / 8);
    const long long need = p->precision == 32 ? FUSED_AUTO_STRIPS_32 : FUSED_AUTO_STRIPS_64;
    c->fused = p->kernel_path >= 2 || (p->kernel_path == 0 && strips8 >= need);
    c->fused_nt = L.state_bytes > FUSED_CACHED_STATE_BYTES;
  }
  {
    // k_step2 strips.  Width: 224 or 240 columns (whole 64-byte segments of
    // a row), whichever leaves fewer of the 256 lanes per row idle (16384^2
    // on MI355X: 240 columns, 5.92 against 6.25 ms per step).  Height: S2_H
    // rows, halved (down to 16) while the launch has fewer than
    // S2_MIN_BLOCKS workgroups; a launch of only a few rounds of resident
    // workgroups takes the height in [S2_ROUND_H_MIN, S2_H] that fills its
    // last round best.
    c->two_step = two_step_of(p, L.state_bytes);
    auto lanes_used = [&](int w) {
      return (double)p->nx / ((double)((p->nx + w - 1) / w) * S2_L);
    };
    c->w2s = lanes_used(240) >= lanes_used(224) ? 240 : 224;
    c->ntx2s = (p->nx + c->w2s - 1) / c->w2s;
    int h = S2_H;
    while (h > 16 && (long long)c->ntx2s * ((p->ny + h - 1) / h) < S2_MIN_BLOCKS) h /= 2;
    int cus = 0;
    if (h >= S2_ROUND_H_MIN &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0) {
      const long long slots = (long long)S2_WG_PER_CU * cus;
      if ((long long)c->ntx2s * ((p->ny + h - 1) / h) < FUSED_FEW_ROUNDS * slots) {
        double best = -1.0;
        int hb = h;
        for (int hh = S2_ROUND_H_MIN; hh <= S2_H; ++hh) {
          const long long n = (long long)c->ntx2s * ((p->ny + hh - 1) / hh);
          if (n < slots) continue;  // at least one full round
          const double eff = (double)n / (double)(((n + slots - 1) / slots) * slots);
          if (eff > best + 1e-9 || (eff > best - 1e-9 && std::abs(hh - h) < std::abs(hb - h))) {
            best = eff;
            hb = hh;
          }
        }
        h = hb;
      }
    }
    c->h2s = h;
    c->nty2s = (p->ny + h - 1) / h;
    c->s2_xcd = (long long)c->ntx2s * c->nty2s < FUSED_DISPATCH_ORDER_BLOCKS_32;
  }
  c->partials = reinterpret_cast<double*>(c->ws);
  c->red_mid = c->partials + (size_t)L.ntx2 * L.nty2 * NQ;
  c->diag_dev = c->red_mid + (size_t)RED_BLOCKS * NQ;
  c->diag_pending = c->diag_seen = c->nonfinite = false;
  c->u0_zero = ux0 == nullptr && uy0 == nullptr;
  c->adj = nullptr;
  c->th_part = c->th_out = nullptr;
  c->timing = false;
  KP& k = c->kp;
  k.nx = p->nx;
  k.ny = p->ny;
  k.pitch = (int)L.pitch;
  k.bcx = p->bc_x;
  k.bcy = p->bc_y;
  k.ps = (long long)L.ps;
  k.phim = 0.5 * (p->phi_A + p->phi_B);
  k.phi_ref = p->precision == 32 ? k.phim : 0.0;
  k.phiA = p->phi_A;
  k.phiB = p->phi_B;
  k.beta4 = 4.0 * d.beta;
  k.kappa = d.kappa;
  k.alpha = d.alpha;
  k.omega_f = 1.0 / d.tau_f;
  k.rhoB = p->rho_B;
  k.rho_slope = (p->rho_A - p->rho_B) / (p->phi_A - p->phi_B);
  k.nuB = d.nu_B;
  k.nu_slope = (d.nu_A - d.nu_B) / (p->phi_A - p->phi_B);
  k.gx = p->gx;
  k.gy = p->gy;
  k.nu_form = p->nu_form;
  k.dphiAB = p->phi_A - p->phi_B;
  k.nuA = d.nu_A;
  k.ln_nuA = std::log(d.nu_A);
  k.ln_nuB = std::log(d.nu_B);
  k.inv_nuA = 1.0 / d.nu_A;
  k.inv_nuB = 1.0 / d.nu_B;
  k.nu_dphi = p->nu_form == LBM_NU_INVERSE ? (k.inv_nuB - k.inv_nuA) / k.dphiAB
                                           : (k.ln_nuA - k.ln_nuB) / k.dphiAB;
  k.collision = p->collision;
  for (int i = 0; i < 4; ++i) k.mf[i] = p->mrt_f[i];
  for (int i = 0; i < 2; ++i) k.mg[i] = p->mrt_g[i];
  // the 16-bit low word of f_0 pays where the step is bound by HBM; on
  // smaller states its arithmetic costs more than the bytes it saves
  c->lo16 = lo16_of(p, L.state_bytes);
  c->d.lo16 = c->lo16 ? 1 : 0;
  c->d.two_step = c->two_step ? 1 : 0;
  hipError_t e = hipHostMalloc((void**)&c->diag_host, (2 * NQ + 6) * sizeof(double), hipHostMallocDefault);
  if (e != hipSuccess) {
    delete c;
    return LBM_EHIP;
  }
  e = hipEventCreateWithFlags(&c->diag_ev, hipEventDisableTiming);
  if (e != hipSuccess) {
    hipHostFree(c->diag_host);
    delete c;
    return LBM_EHIP;
  }
  r = c->prec == 64 ? init_impl<double>(c, phi0, ux0, uy0) : init_impl<float>(c, phi0, ux0, uy0);
  if (r) {
    lbm_destroy(c);
    return r;
  }
  *out = c;
  return LBM_OK;
}

int lbm_step(lbm_ctx* c, int64_t n) {
  if (!c) return LBM_EINVAL;
  if (n < 0) return LBM_EINVAL;
  int r = consume_diag(c, false);
  if (r) return r;
  if (c->nonfinite) return LBM_ENONFINITE;
  r = c->prec == 64 ? step_impl<double>(c, n) : step_impl<float>(c, n);
  if (r) return r;
  r = consume_diag(c, false);
  if (r) return r;
  return c->nonfinite ? LBM_ENONFINITE : LBM_OK;
}

int lbm_step_noalloc(lbm_ctx* c, int64_t n) {
  if (!c) return LBM_EINVAL;
  if (n < 0) return LBM_EINVAL;
  if (c->timing) {
    c->err = "lbm_step_noalloc: step timing records new events; stop it (lbm_timing 0) first";
    return LBM_ESTATE;
  }
  if (!c->scratch_dev) {
    c->err = std::string("lbm_step_noalloc: no scratch on this device: hipGetSymbolAddress: ") +
             hipGetErrorString(c->scratch_err);
    return LBM_EHIP;
  }
  // the step's diagnostic partials (one per strip or tile), the first-level
  // reduction and the reduced diagnostics, laid out as in the workspace
  const long long nparts = step_partials(c);
  const size_t need = ((size_t)nparts * NQ + (size_t)RED_BLOCKS * NQ + NQ) * sizeof(double);
  if (c->p.diag_every > 0 && need > NOALLOC_SCRATCH_BYTES) {
    c->err = "lbm_step_noalloc: the diagnostics of this grid need " + std::to_string(need) +
             " bytes of scratch, above its " + std::to_string(NOALLOC_SCRATCH_BYTES) + " bytes";
    return LBM_EINVAL;
  }
  // every kernel below writes these before it reads them: nothing to clear
  double* const keep[3] = {c->partials, c->red_mid, c->diag_dev};
  c->partials = c->scratch_dev;
  c->red_mid = c->partials + (size_t)nparts * NQ;
  c->diag_dev = c->red_mid + (size_t)RED_BLOCKS * NQ;
  const int r = lbm_step(c, n);
  c->partials = keep[0];
  c->red_mid = keep[1];
  c->diag_dev = keep[2];
  return r;
}

int64_t lbm_step_count(const lbm_ctx* c) { return c ? c->step : -1; }

int lbm_moments(lbm_ctx* c, double* phi, double* mu, double* ux, double* uy, double* p,
                double* rho, lbm_diag* diag) {
  if (!c) return LBM_EINVAL;
  MomOut mo{phi, mu, ux, uy, p, rho};
  return c->prec == 64 ? moments_impl<double>(c, mo, diag) : moments_impl<float>(c, mo, diag);
}

int lbm_last_diag(lbm_ctx* c, lbm_diag* diag) {
  if (!c || !diag) return LBM_EINVAL;
  int r = consume_diag(c, true);
  if (r) return r;
  if (!c->diag_seen) return LBM_ESTATE;
  fill_diag(c->diag_host, c->diag_step, diag, nullptr);
  return diag_bad(c->diag_host) ? LBM_ENONFINITE : LBM_OK;
}

int lbm_get_state(lbm_ctx* c, int32_t x0, int32_t y0, int32_t w, int32_t h, double* f, double* g,
                  double* Sp) {
  if (!c) return LBM_EINVAL;
  if (w < 1 || h < 1 || w > c->p.nx || h > c->p.ny) return LBM_EINVAL;
  x0 = ((x0 % c->p.nx) + c->p.nx) % c->p.nx;
  y0 = ((y0 % c->p.ny) + c->p.ny) % c->p.ny;
  return c->prec == 64 ? get_state_impl<double>(c, x0, y0, w, h, f, g, Sp)
                       : get_state_impl<float>(c, x0, y0, w, h, f, g, Sp);
}

int lbm_set_state(lbm_ctx* c, const double* f, const double* g, const double* Sp, int64_t step) {
  if (!c || !f || !g || !Sp || step < 0) return LBM_EINVAL;
  int r = c->prec == 64 ? set_state_impl<double>(c, f, g, Sp) : set_state_impl<float>(c, f, g, Sp);
  if (r) return r;
  c->step = step;
  c->nonfinite = false;
  return LBM_OK;
}

int lbm_timing(lbm_ctx* c, int enable) {
  if (!c) return LBM_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  for (hipEvent_t e : c->tev) hipEventDestroy(e);
  c->tev.clear();
  c->tev_steps.clear();
  c->timing = enable != 0;
  return LBM_OK;
}

int lbm_kernel_times(lbm_ctx* c, double* ms_step, int64_t* steps) {
  if (!c) return LBM_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  double a = 0.0;
  for (size_t k = 0; k + 1 < c->tev.size(); k += 2) {
    float t = 0.f;
    HIPCHK(c, hipEventElapsedTime(&t, c->tev[k], c->tev[k + 1]));
    a += t;
  }
  if (ms_step) *ms_step = a;
  int64_t ns = 0;
  for (int k : c->tev_steps) ns += k;
  if (steps) *steps = ns;
  return LBM_OK;
}

int lbm_stream_copy(void* dst, const void* src, size_t bytes, void* stream) {
  if (!dst || !src || (bytes & 15) || ((uintptr_t)dst & 15) || ((uintptr_t)src & 15))
    return LBM_EINVAL;
  const long long n = (long long)(bytes / 16);
  if (n == 0) return LBM_OK;
  long long blocks = (n + 255) / 256;
  if (blocks > 256 * 1024) blocks = 256 * 1024;
  hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, static_cast<hipStream_t>(stream),
                     static_cast<float4*>(dst), static_cast<const float4*>(src), n);
  return hipGetLastError() == hipSuccess ? LBM_OK : LBM_EHIP;
}

size_t lbm_adjoint_workspace_bytes(const lbm_params* p) {
  if (validate(p, nullptr) != LBM_OK) return 0;
  return adj_bytes(p);
}

int lbm_adjoint_attach(lbm_ctx* c, void* adj_workspace) {
  if (!c || !adj_workspace || ((uintptr_t)adj_workspace & 255)) return LBM_EINVAL;
  c->adj = static_cast<char*>(adj_workspace);
  c->th_part = reinterpret_cast<double*>(c->adj + ADJ_PLANES * adj_plane_bytes(&c->p));
  const long long tiles = (long long)th_tiles(&c->p);
  c->th_out = c->th_part + tiles * NTH;
  hipLaunchKernelGGL(k_zero, dim3(256), dim3(256), 0, c->stream, c->th_part, (tiles + 1) * NTH);
  LAUNCHCHK(c);
  return LBM_OK;
}

int lbm_step_into(lbm_ctx* c, void* src, void* dst) {
  if (!c || !src || !dst || src == dst) return LBM_EINVAL;
  if (((uintptr_t)src & 255) || ((uintptr_t)dst & 255)) return LBM_EINVAL;
  return c->prec == 64 ? step_into_impl<double>(c, static_cast<double*>(src), static_cast<double*>(dst))
                       : step_into_impl<float>(c, static_cast<float*>(src), static_cast<float*>(dst));
}

int lbm_adjoint_step(lbm_ctx* c, void* state, const void* lam_in, void* lam_out, int flags) {
  if (!c || !state || !lam_in || !lam_out || lam_in == lam_out) return LBM_EINVAL;
  if (((uintptr_t)state & 255) || (flags & ~LBM_SNAPSHOT_HAS_PHI_MU)) return LBM_EINVAL;
  if (!c->adj) return LBM_ESTATE;
  const bool have = (flags & LBM_SNAPSHOT_HAS_PHI_MU) != 0;
  return c->prec == 64 ? adjoint_step_impl<double>(c, static_cast<double*>(state),
                                                   static_cast<const double*>(lam_in),
                                                   static_cast<double*>(lam_out), have)
                       : adjoint_step_impl<float>(c, static_cast<float*>(state), static_cast<const float*>(lam_in),
                                                  static_cast<float*>(lam_out), have);
}

int lbm_adjoint_segment(lbm_ctx* c, void* const* snaps, int L, void* lam, void* tmp, int* which) {
  if (!c || !snaps || L < 1 || !lam || !tmp || !which || lam == tmp) return LBM_EINVAL;
  for (int k = 0; k < L; ++k)
    if (!snaps[k] || ((uintptr_t)snaps[k] & 255)) return LBM_EINVAL;
  if (!c->adj) return LBM_ESTATE;
  return c->prec == 64 ? adjoint_segment_impl<double>(c, reinterpret_cast<double* const*>(snaps), L,
                                                      static_cast<double*>(lam), static_cast<double*>(tmp), which)
                       : adjoint_segment_impl<float>(c, reinterpret_cast<float* const*>(snaps), L,
                                                     static_cast<float*>(lam), static_cast<float*>(tmp), which);
}

int lbm_adjoint_init(lbm_ctx* c, const void* state, const double* phi0, const void* lam0, void* scratch,
                     double* dphi0) {
  if (!c || !state || !phi0 || !lam0 || !scratch || !dphi0 || lam0 == scratch) return LBM_EINVAL;
  if ((uintptr_t)state & 255) return LBM_EINVAL;
  if (!c->adj || !c->u0_zero) return LBM_ESTATE;
  return c->prec == 64
             ? adjoint_init_impl<double>(c, static_cast<const double*>(state), phi0,
                                         static_cast<const double*>(lam0), static_cast<double*>(scratch), dphi0)
             : adjoint_init_impl<float>(c, static_cast<const float*>(state), phi0, static_cast<const float*>(lam0),
                                        static_cast<float*>(scratch), dphi0);
}

int lbm_adjoint_theta(lbm_ctx* c, int basis, double* out, int reset) {
  if (!c || !out || (basis != LBM_THETA_NATIVE && basis != LBM_THETA_TAU)) return LBM_EINVAL;
  if (!c->adj) return LBM_ESTATE;
  const long long tiles = (long long)th_tiles(&c->p);
  hipLaunchKernelGGL(k_sum_theta, dim3(1), dim3(256), 0, c->stream, c->th_part, tiles, c->th_out);
  LAUNCHCHK(c);
  HIPCHK(c, hipMemcpyAsync(out, c->th_out, NTH * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (basis == LBM_THETA_TAU) {
    // from (kappa, beta, alpha, tau_f, nu_A, nu_B) to (kappa, beta, M,
    // tau_f, tau_gA, tau_gB): alpha = M / (c_s^2 (tau_f - 1/2)) (eq.
    // mobility), so d alpha/d M = alpha / M and d alpha/d tau_f at fixed M
    // = -alpha / (tau_f - 1/2); nu = c_s^2 (tau_g - 1/2) (Sec. 2.3.2)
    const double a = c->d.alpha, tf = c->d.tau_f, ga = out[2], gt = out[3];
    out[2] = ga * (a / c->p.M);
    out[3] = gt - ga * (a / (tf - 0.5));
    out[4] *= CS2;
    out[5] *= CS2;
  }
  if (reset) {
    hipLaunchKernelGGL(k_zero, dim3(256), dim3(256), 0, c->stream, c->th_part, tiles * NTH);
    LAUNCHCHK(c);
  }
  return LBM_OK;
}

size_t lbm_snapshot_bytes(const lbm_ctx* c) { return c ? snapshot_bytes(c) : 0; }

int lbm_snapshot(lbm_ctx* c, void* dst) {
  if (!c || !dst) return LBM_EINVAL;
  const size_t pb = (size_t)c->kp.ps * c->esz;
  const size_t nb = c->prec == 64 ? Store<double>::NB : Store<float>::NB;
  char* base = c->state + (size_t)c->cur * nb * pb;
  HIPCHK(c, hipMemcpyAsync(dst, base, nb * pb, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(static_cast<char*>(dst) + nb * pb, c->state + (2 * nb + c->scur) * pb, pb,
                           hipMemcpyDeviceToDevice, c->stream));
  return LBM_OK;
}

int lbm_restore(lbm_ctx* c, const void* src, int64_t step) {
  if (!c || !src || step < 0) return LBM_EINVAL;
  const size_t pb = (size_t)c->kp.ps * c->esz;
  const size_t nb = c->prec == 64 ? Store<double>::NB : Store<float>::NB;
  char* base = c->state + (size_t)c->cur * nb * pb;
  HIPCHK(c, hipMemcpyAsync(base, src, nb * pb, hipMemcpyDeviceToDevice, c->stream));
  HIPCHK(c, hipMemcpyAsync(c->state + (2 * nb + c->scur) * pb, static_cast<const char*>(src) + nb * pb, pb,
                           hipMemcpyDeviceToDevice, c->stream));
  c->step = step;
  c->nonfinite = false;
  return LBM_OK;
}

int lbm_destroy(lbm_ctx* c) {
  if (!c) return LBM_OK;
  hipStreamSynchronize(c->stream);
  for (hipEvent_t e : c->tev) hipEventDestroy(e);
  if (c->diag_ev) hipEventDestroy(c->diag_ev);
  if (c->diag_host) hipHostFree(c->diag_host);
  delete c;
  return LBM_OK;
}

const char* lbm_strerror(int code) {
  switch (code) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument";
    case LBM_EHIP: return "HIP runtime error";
    case LBM_ENONFINITE: return "non-finite value or non-positive density in diagnostics";
    case LBM_ESTATE: return "call made in the wrong state";
    default: return "unknown error";
  }
}

const char* lbm_last_error(const lbm_ctx* c) { return c ? c->err.c_str() : ""; }

}  // extern "C"
