// HIP kernels and C ABI of the well-balanced phase-field LBM step for
// MI355X (gfx950).  The operations each kernel performs are cited from the
// paper (Ju et al., arXiv 2311.10827) next to the code; the ABI contract is
// in include/lbmwb.h.
//
// Data layout in HBM (all planes of the storage type T, 256-byte aligned):
//   state = [pop buffer 0: 18 planes][pop buffer 1: 18 planes][S][dphi][mu]
//   pop planes 0..8 hold f_i, 9..17 hold g_i, row-major [ny][pitch].
// A pop buffer holds the post-collision values of the previous step; the
// pre-collision population of the current step is their pull gather
//   f_i(x) = B_i(x - c_i)        if the link from x - c_i is fluid,
//   f_i(x) = B_opp(i)(x)         if it crosses a wall (half-way bounce-back).
// Each step reads one buffer and writes the other.  The dphi plane holds
// phi - phi_ref and the f_0 plane holds f_0 - phi_ref (phi_ref = 0 in FP64,
// (phi_A + phi_B)/2 in FP32), so FP32 storage keeps the full precision of
// the small deviations that carry the force balance.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "lbmwb.h"

namespace {

// ------------------------------------------------------------------ lattice
// D2Q9 (Sec. 2.2, eq. eq:ci): 0 rest, 1 E, 2 N, 3 W, 4 S, 5 NE, 6 NW, 7 SW, 8 SE.
__host__ __device__ constexpr int cx_of(int i) {
  return (i == 1 || i == 5 || i == 8) ? 1 : (i == 3 || i == 6 || i == 7) ? -1 : 0;
}
__host__ __device__ constexpr int cy_of(int i) {
  return (i == 2 || i == 5 || i == 6) ? 1 : (i == 4 || i == 7 || i == 8) ? -1 : 0;
}
__host__ __device__ constexpr int opp_of(int i) {
  return i == 0 ? 0 : (i <= 4 ? ((i + 1) % 4) + 1 : ((i - 3) % 4) + 5);
}
// weights w_i (Sec. 2.2, after eq. H_iyang)
__host__ __device__ constexpr double w_of(int i) {
  return i == 0 ? 4.0 / 9.0 : (i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0);
}
// Convection source shape: w_i [-1 + I:(c_i c_i - c_s^2 I)/(2 c_s^2)] (Sec. 2.3.1, eq. F_i)
// = w_i (3/2 |c_i|^2 - 2): -8/9 rest, -1/18 axis, +1/36 diagonal.
__host__ __device__ constexpr double src_of(int i) {
  return i == 0 ? -8.0 / 9.0 : (i <= 4 ? -1.0 / 18.0 : 1.0 / 36.0);
}

constexpr int NPOP = 18;
constexpr int NQ = 11;  // diagnostic quantities, order of lbm_diag's leading fields

// Kernel parameters: geometry plus constants of the step, in FP64 (each
// kernel converts them once to its compute type).
struct KP {
  int nx, ny, pitch, bcx, bcy;
  long long ps;        // plane stride in elements
  double phi_ref;      // stored offset of phi and f_0
  double cA, cB;       // phi_ref - phi_A, phi_ref - phi_B: (phi - phi_A) = dphi + cA
  double beta4;        // 4 beta
  double kappa, alpha;
  double omega_f;      // 1 / tau_f
  double rhoB, drho;   // rho = rho_B + (phi - phi_B) drho
  double tgB, dtg;     // tau_g = tau_gB + (phi - phi_B) dtg
  double gx, gy;
};

// XCD-aware tile order: the hardware deals workgroups round-robin over the
// 8 XCDs, so give each XCD one contiguous band of tiles; neighbouring tiles
// then share that XCD's L2.
__device__ __forceinline__ int xcd_tile(int b, int n) {
  const int X = 8;
  const int per = n / X, rem = n % X;
  const int xcd = b % X, local = b / X;
  return xcd < rem ? xcd * (per + 1) + local : rem * (per + 1) + (xcd - rem) * per + local;
}

// Stencil neighbour index: periodic wrap, or the mirrored adjacent cell
// across a wall.  Valid for any integer v (tiles may overhang the grid).
__device__ __forceinline__ int stencil_idx(int v, int n, int wall) {
  if (wall) return v < 0 ? 0 : (v >= n ? n - 1 : v);
  int r = v % n;
  return r < 0 ? r + n : r;
}

// Pull source of the link that arrives at v along +1 (d = +1: source v-1)
// or -1 (source v+1); -1 marks a link that crosses a wall.
struct PullCols {
  int m, p;  // source for c = +1 (i.e. v-1) and for c = -1 (v+1)
};
__device__ __forceinline__ PullCols pull_cols(int v, int n, int wall) {
  PullCols r;
  r.m = v > 0 ? v - 1 : (wall ? -1 : n - 1);
  r.p = v < n - 1 ? v + 1 : (wall ? -1 : 0);
  return r;
}

// NP = 9 gathers f only, NP = 18 gathers f and g.
template <int NP = NPOP, typename T>
__device__ __forceinline__ void gather_pops(const T* __restrict__ B, const KP& p, int x, int y,
                                            T (&pop)[NP]) {
  const PullCols px = pull_cols(x, p.nx, p.bcx);
  const PullCols py = pull_cols(y, p.ny, p.bcy);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int cx = cx_of(i), cy = cy_of(i);
    const int sx = cx == 1 ? px.m : (cx == -1 ? px.p : x);
    const int sy = cy == 1 ? py.m : (cy == -1 ? py.p : y);
    long long off;
    int plane;
    if (sx < 0 || sy < 0) {  // half-way bounce-back
      plane = opp_of(i);
      off = (long long)y * p.pitch + x;
    } else {
      plane = i;
      off = (long long)sy * p.pitch + sx;
    }
    pop[i] = B[plane * p.ps + off];
    if (NP == NPOP) pop[(9 + i) % NP] = B[(9 + plane) * p.ps + off];
  }
}

// ------------------------------------------------------------ diagnostics
struct Diag {
  double v[NQ];
};
__device__ __forceinline__ void diag_identity(Diag& d) {
  d.v[0] = d.v[1] = d.v[2] = 0.0;
  d.v[3] = 0.0;
  d.v[4] = INFINITY;
  d.v[5] = -INFINITY;
  d.v[6] = INFINITY;
  d.v[7] = -INFINITY;
  d.v[8] = INFINITY;
  d.v[9] = -INFINITY;
  d.v[10] = 0.0;
}
__host__ __device__ inline bool diag_is_min(int k) { return k == 4 || k == 6 || k == 8; }
__host__ __device__ inline bool diag_is_max(int k) { return k == 3 || k == 5 || k == 7 || k == 9; }
__device__ __forceinline__ double diag_op(int k, double a, double b) {
  return diag_is_min(k) ? fmin(a, b) : (diag_is_max(k) ? fmax(a, b) : a + b);
}

// Block reduction in a fixed order: xor-butterfly within each 64-lane
// wavefront, then waves in index order.  Bitwise reproducible.
__device__ void block_reduce_write(Diag& d, double* __restrict__ out) {
  __shared__ double red[4][NQ];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NQ; ++k) {
    double a = d.v[k];
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) a = diag_op(k, a, __shfl_xor(a, s, 64));
    d.v[k] = a;
  }
  if (lane == 0)
    for (int k = 0; k < NQ; ++k) red[wave][k] = d.v[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = blockDim.x >> 6;
    for (int k = 0; k < NQ; ++k) {
      double a = red[0][k];
      for (int w = 1; w < nw; ++w) a = diag_op(k, a, red[w][k]);
      out[k] = a;
    }
  }
}

__global__ __launch_bounds__(256) void k_reduce_diag(const double* __restrict__ partials, int n,
                                                      double* __restrict__ out) {
  Diag d;
  diag_identity(d);
  for (int b = threadIdx.x; b < n; b += blockDim.x)
    for (int k = 0; k < NQ; ++k) d.v[k] = diag_op(k, d.v[k], partials[(long long)b * NQ + k]);
  block_reduce_write(d, out);
}

// -------------------------------------------------------- phi / mu stencil
// phi = sum_i f_i (Sec. 2.3.1, eq. order-parameter) on a tile plus a one-cell
// ring, staged in LDS; then mu = 4 beta (phi - phi_A)(phi - phi_B)(phi - phi_m)
// - kappa lap(phi) (Sec. 2.1, eq. chemical_potencial) with the isotropic
// Laplacian lap = sum_{i!=0} 2 w_i [phi(x + c_i) - phi(x)] / c_s^2
// (Sec. 2.3.2, eq. Laplace) in its difference form.
// FROM_INPUT: phi comes from the caller's FP64 field (initialisation).
constexpr int K1_TX = 64, K1_TY = 16;

template <typename T, bool FROM_INPUT>
__global__ __launch_bounds__(256) void k_phi_mu(const KP p, const T* __restrict__ B,
                                                 const double* __restrict__ phi_in,
                                                 T* __restrict__ dphi_out, T* __restrict__ mu_out,
                                                 int ntx) {
  using C = typename std::conditional<FROM_INPUT, double, T>::type;
  constexpr int LW = K1_TX + 2, LH = K1_TY + 2;
  __shared__ C s[LH * LW];
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int x0 = (tile % ntx) * K1_TX, y0 = (tile / ntx) * K1_TY;
  for (int k = threadIdx.x; k < LH * LW; k += blockDim.x) {
    const int ly = k / LW, lx = k - ly * LW;
    const int gx = stencil_idx(x0 + lx - 1, p.nx, p.bcx);
    const int gy = stencil_idx(y0 + ly - 1, p.ny, p.bcy);
    C v;
    if (FROM_INPUT) {
      v = (C)(phi_in[(long long)gy * p.nx + gx] - p.phi_ref);
    } else {
      T pop[9];
      gather_pops<9>(B, p, gx, gy, pop);
      v = pop[0] + (((pop[1] + pop[2]) + (pop[3] + pop[4])) + ((pop[5] + pop[6]) + (pop[7] + pop[8])));
    }
    s[k] = v;
  }
  __syncthreads();
  const C beta4 = (C)p.beta4, kappa = (C)p.kappa, cA = (C)p.cA, cB = (C)p.cB;
  const int lx = threadIdx.x % K1_TX;
  for (int ly = threadIdx.x / K1_TX; ly < K1_TY; ly += blockDim.x / K1_TX) {
    const int x = x0 + lx, y = y0 + ly;
    if (x >= p.nx || y >= p.ny) continue;
    const C* r0 = s + ly * LW + lx;  // row y-1, column x-1
    const C* r1 = r0 + LW;
    const C* r2 = r1 + LW;
    const C c = r1[1];
    const C axis = ((r1[2] - c) + (r1[0] - c)) + ((r2[1] - c) + (r0[1] - c));
    const C diag = ((r2[2] - c) + (r2[0] - c)) + ((r0[2] - c) + (r0[0] - c));
    const C lap = (C)(2.0 / 3.0) * axis + (C)(1.0 / 6.0) * diag;
    // phi - phi_m = dphi + (phi_ref - phi_m); phi_ref is phi_m or 0
    const C dm = c + (C)(0.5 * (p.cA + p.cB));
    const C mu = beta4 * ((c + cA) * (c + cB)) * dm - kappa * lap;
    const long long o = (long long)y * p.pitch + x;
    dphi_out[o] = (T)c;
    mu_out[o] = (T)mu;
  }
}

// ---------------------------------------------------- fused collide-stream
// For every cell: gather f_i, g_i (pull streaming with bounce-back), read
// the 3x3 neighbourhoods of phi and mu, then
//   grad phi, grad mu by the isotropic stencil (Sec. 2.3.2, eq. gradient);
//   rho, tau_g linear in phi (Sec. 2.3.2, eq. vis), grad rho = drho grad phi;
//   F = -phi grad mu + G (Sec. 2.1 after eq. 6; Sec. 2.3.2 after eq. GGi);
//   rho u = sum c_i g_i + F/2, p = c_s^2/(1-w_0) [sum_{i!=0} g_i + u.grad(rho)/2
//     + rho s_0(u)] (Sec. 2.3.2, macroscopic subequations);
//   S = u.grad phi; f collision with F_i(S) + [F_i(S) - F_i(S_prev)]/2
//     (Sec. 2.3.1, eqs. BGK, H_i, F_i; backward difference for the time
//     derivative);
//   g collision with g^eq and G_i (Sec. 2.3.2, eqs. BGK-NS, G_i, Siu, GGi;
//     G_i = (1 - 1/(2 tau_g)) 3 w_i [c_i.F + (c_i.u)(c_i.grad rho)]).
enum Mode { M_STEP = 0, M_STEP_DIAG = 1, M_MOMENTS = 2, M_INIT_S = 3 };

struct MomOut {
  double *phi, *mu, *ux, *uy, *p, *rho;
};

constexpr int K2_TX = 64, K2_TY = 4;

template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_collide(const KP p, const T* __restrict__ Bin,
                                                  T* __restrict__ Bout, T* __restrict__ Spl,
                                                  const T* __restrict__ dphi,
                                                  const T* __restrict__ mupl, MomOut mo,
                                                  double* __restrict__ partials, int ntx) {
  constexpr bool DIAG = MODE == M_STEP_DIAG || MODE == M_MOMENTS;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int x = (tile % ntx) * K2_TX + (threadIdx.x & (K2_TX - 1));
  const int y = (tile / ntx) * K2_TY + threadIdx.x / K2_TX;
  const bool valid = x < p.nx && y < p.ny;
  Diag dg;
  if (DIAG) diag_identity(dg);
  if (valid) {
    const long long o = (long long)y * p.pitch + x;
    T pop[NPOP];
    gather_pops(Bin, p, x, y, pop);
    // 3x3 neighbourhoods, rows y-1, y, y+1 and columns x-1, x, x+1
    const int xm = stencil_idx(x - 1, p.nx, p.bcx), xp = stencil_idx(x + 1, p.nx, p.bcx);
    const int ym = stencil_idx(y - 1, p.ny, p.bcy), yp = stencil_idx(y + 1, p.ny, p.bcy);
    const long long rm = (long long)ym * p.pitch, r0 = (long long)y * p.pitch,
                    rp = (long long)yp * p.pitch;
    T ph[3][3], m[3][3];
    ph[0][0] = dphi[rm + xm]; ph[0][1] = dphi[rm + x]; ph[0][2] = dphi[rm + xp];
    ph[1][0] = dphi[r0 + xm]; ph[1][1] = dphi[r0 + x]; ph[1][2] = dphi[r0 + xp];
    ph[2][0] = dphi[rp + xm]; ph[2][1] = dphi[rp + x]; ph[2][2] = dphi[rp + xp];
    m[0][0] = mupl[rm + xm]; m[0][1] = mupl[rm + x]; m[0][2] = mupl[rm + xp];
    m[1][0] = mupl[r0 + xm]; m[1][1] = mupl[r0 + x]; m[1][2] = mupl[r0 + xp];
    m[2][0] = mupl[rp + xm]; m[2][1] = mupl[rp + x]; m[2][2] = mupl[rp + xp];
    const T third = (T)(1.0 / 3.0), twelfth = (T)(1.0 / 12.0);
    const T gpx = third * (ph[1][2] - ph[1][0]) + twelfth * ((ph[2][2] - ph[2][0]) + (ph[0][2] - ph[0][0]));
    const T gpy = third * (ph[2][1] - ph[0][1]) + twelfth * ((ph[2][2] - ph[0][2]) + (ph[2][0] - ph[0][0]));
    const T gmx = third * (m[1][2] - m[1][0]) + twelfth * ((m[2][2] - m[2][0]) + (m[0][2] - m[0][0]));
    const T gmy = third * (m[2][1] - m[0][1]) + twelfth * ((m[2][2] - m[0][2]) + (m[2][0] - m[0][0]));
    const T dph = ph[1][1];               // phi - phi_ref
    const T phi = dph + (T)p.phi_ref;
    const T mu = m[1][1];
    const T dB = dph + (T)p.cB;           // phi - phi_B
    const T drho = (T)p.drho;
    const T rho = (T)p.rhoB + dB * drho;
    const T grx = drho * gpx, gry = drho * gpy;
    const T Fx = (T)p.gx - phi * gmx, Fy = (T)p.gy - phi * gmy;
    const T* g = pop + 9;
    const T mx = ((g[1] - g[3]) + (g[5] - g[7])) + (g[8] - g[6]);
    const T my = ((g[2] - g[4]) + (g[5] - g[7])) + (g[6] - g[8]);
    const T gnz = ((g[1] + g[2]) + (g[3] + g[4])) + ((g[5] + g[6]) + (g[7] + g[8]));
    const T irho = (T)1 / rho;
    const T ux = (mx + (T)0.5 * Fx) * irho, uy = (my + (T)0.5 * Fy) * irho;
    const T uu = ux * ux + uy * uy;
    const T ugr = ux * grx + uy * gry;
    const T pr = (T)0.6 * (gnz + (T)0.5 * ugr - (T)(2.0 / 3.0) * rho * uu);
    const T S = ux * gpx + uy * gpy;

    if (MODE == M_MOMENTS) {
      if (mo.phi) mo.phi[(long long)y * p.nx + x] = (double)dph + p.phi_ref;
      if (mo.mu) mo.mu[(long long)y * p.nx + x] = (double)mu;
      if (mo.ux) mo.ux[(long long)y * p.nx + x] = (double)ux;
      if (mo.uy) mo.uy[(long long)y * p.nx + x] = (double)uy;
      if (mo.p) mo.p[(long long)y * p.nx + x] = (double)pr;
      if (mo.rho) mo.rho[(long long)y * p.nx + x] = (double)rho;
    }
    const T Sp = Spl[o];
    if (MODE == M_INIT_S) Spl[o] = S;
    if (MODE == M_STEP || MODE == M_STEP_DIAG) {
      // order-parameter population (stored f_0 is f_0 - phi_ref)
      const T src = (T)1.5 * S - (T)0.5 * Sp;
      const T wf = (T)p.omega_f;
      const T am = (T)p.alpha * mu;
      const T* f = pop;
      Bout[o] = f[0] + wf * ((dph - (T)(5.0 / 9.0) * am) - f[0]) + (T)src_of(0) * src;
#pragma unroll
      for (int i = 1; i < 9; ++i)
        Bout[i * p.ps + o] = f[i] + wf * ((T)w_of(i) * am - f[i]) + (T)src_of(i) * src;
      // hydrodynamic population
      const T tg = (T)p.tgB + dB * (T)p.dtg;
      const T wg = (T)1 / tg;
      const T kG = (T)1 - (T)0.5 * wg;
      const T ge0 = -(T)(5.0 / 3.0) * pr - (T)(2.0 / 3.0) * rho * uu;
      Bout[9 * p.ps + o] = g[0] + wg * (ge0 - g[0]);
      const T p3 = (T)3 * pr, ruu = (T)1.5 * rho * uu;
#pragma unroll
      for (int i = 1; i < 9; ++i) {
        const T cu = (T)cx_of(i) * ux + (T)cy_of(i) * uy;
        const T cF = (T)cx_of(i) * Fx + (T)cy_of(i) * Fy;
        const T cr = (T)cx_of(i) * grx + (T)cy_of(i) * gry;
        const T w = (T)w_of(i);
        const T geq = w * (p3 + rho * (cu * ((T)3 + (T)4.5 * cu)) - ruu);
        const T Gi = kG * (T)3 * w * (cF + cu * cr);
        Bout[(9 + i) * p.ps + o] = g[i] + wg * (geq - g[i]) + Gi;
      }
      Spl[o] = S;
    }
    if (DIAG) {
      const double dphi_d = (double)dph + p.phi_ref;
      const bool fin = isfinite((double)phi) && isfinite((double)mu) && isfinite((double)ux) &&
                       isfinite((double)uy) && isfinite((double)pr);
      dg.v[0] = dphi_d;
      dg.v[1] = 1.5 * (double)S - 0.5 * (double)Sp;
      dg.v[2] = 0.5 * (double)rho * ((double)ux * (double)ux + (double)uy * (double)uy);
      dg.v[3] = sqrt((double)ux * (double)ux + (double)uy * (double)uy);
      dg.v[4] = dg.v[5] = (double)rho;
      dg.v[6] = dg.v[7] = (double)mu;
      dg.v[8] = dg.v[9] = dphi_d;
      dg.v[10] = fin ? 0.0 : 1.0;
    }
  }
  if (DIAG) block_reduce_write(dg, partials + (long long)tile * NQ);
}

// ------------------------------------------------------------ state I/O
// Write pre-collision populations into a pop buffer as the values whose pull
// gather returns them: f_i(x) is stored at B_i(x - c_i), or at B_opp(i)(x)
// if the link crosses a wall.  Every buffer entry is written exactly once.
template <typename T>
__device__ __forceinline__ void scatter_pop(T* __restrict__ B, const KP& p, int x, int y, int plane0,
                                            int i, T v) {
  const PullCols px = pull_cols(x, p.nx, p.bcx);
  const PullCols py = pull_cols(y, p.ny, p.bcy);
  const int cx = cx_of(i), cy = cy_of(i);
  const int sx = cx == 1 ? px.m : (cx == -1 ? px.p : x);
  const int sy = cy == 1 ? py.m : (cy == -1 ? py.p : y);
  if (sx < 0 || sy < 0)
    B[(plane0 + opp_of(i)) * p.ps + (long long)y * p.pitch + x] = v;
  else
    B[(plane0 + i) * p.ps + (long long)sy * p.pitch + sx] = v;
}

// Initial populations: f = f^eq(phi0, mu0) (Sec. 2.3.1, eq. H_i) and
// g = g^eq(p = 0, u0) (Sec. 2.3.2, eqs. G_i, Siu); mu0 from k_phi_mu<FROM_INPUT>.
template <typename T>
__global__ __launch_bounds__(256) void k_init_pops(const KP p, T* __restrict__ B,
                                                    const double* __restrict__ phi0,
                                                    const double* __restrict__ ux0,
                                                    const double* __restrict__ uy0,
                                                    const T* __restrict__ mupl) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (long long)p.nx * p.ny) return;
  const int y = (int)(k / p.nx), x = (int)(k - (long long)y * p.nx);
  const double ph = phi0[k];
  const double am = p.alpha * (double)mupl[(long long)y * p.pitch + x];
  scatter_pop<T>(B, p, x, y, 0, 0, (T)((ph - p.phi_ref) - (5.0 / 9.0) * am));
  for (int i = 1; i < 9; ++i) scatter_pop<T>(B, p, x, y, 0, i, (T)(w_of(i) * am));
  const double ux = ux0 ? ux0[k] : 0.0, uy = uy0 ? uy0[k] : 0.0;
  const double rho = p.rhoB + (ph - p.phi_ref + p.cB) * p.drho;
  const double uu = ux * ux + uy * uy;
  scatter_pop<T>(B, p, x, y, 9, 0, (T)(-(2.0 / 3.0) * rho * uu));
  for (int i = 1; i < 9; ++i) {
    const double cu = cx_of(i) * ux + cy_of(i) * uy;
    scatter_pop<T>(B, p, x, y, 9, i, (T)(w_of(i) * rho * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu)));
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_set_state(const KP p, T* __restrict__ B, T* __restrict__ Spl,
                                                    const double* __restrict__ f,
                                                    const double* __restrict__ g,
                                                    const double* __restrict__ Sp) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long n = (long long)p.nx * p.ny;
  if (k >= n) return;
  const int y = (int)(k / p.nx), x = (int)(k - (long long)y * p.nx);
  for (int i = 0; i < 9; ++i) {
    const double v = f[i * n + k] - (i == 0 ? p.phi_ref : 0.0);
    scatter_pop<T>(B, p, x, y, 0, i, (T)v);
    scatter_pop<T>(B, p, x, y, 9, i, (T)g[i * n + k]);
  }
  Spl[(long long)y * p.pitch + x] = (T)Sp[k];
}

template <typename T>
__global__ __launch_bounds__(256) void k_get_state(const KP p, const T* __restrict__ B,
                                                    const T* __restrict__ Spl, int x0, int y0,
                                                    int w, int h, double* __restrict__ f,
                                                    double* __restrict__ g,
                                                    double* __restrict__ Sp) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long n = (long long)w * h;
  if (k >= n) return;
  const int wy = (int)(k / w), wx = (int)(k - (long long)wy * w);
  const int x = (x0 + wx) % p.nx, y = (y0 + wy) % p.ny;
  T pop[NPOP];
  gather_pops(B, p, x, y, pop);
  for (int i = 0; i < 9; ++i) {
    if (f) f[i * n + k] = (double)pop[i] + (i == 0 ? p.phi_ref : 0.0);
    if (g) g[i * n + k] = (double)pop[9 + i];
  }
  if (Sp) Sp[k] = (double)Spl[(long long)y * p.pitch + x];
}

__global__ __launch_bounds__(256) void k_copy(float4* __restrict__ dst, const float4* __restrict__ src,
                                               long long n) {
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x)
    dst[k] = src[k];
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
  int64_t step;
  int ntx1, nty1, ntx2, nty2;
  double* partials;
  double* diag_dev;     // [2][NQ]: fused step diagnostics, moments diagnostics
  double* diag_host;    // pinned [2][NQ]
  int64_t diag_step;
  bool diag_pending, diag_seen, nonfinite;
  hipEvent_t diag_ev;
  bool timing;
  std::vector<hipEvent_t> tev;  // three events per timed step
  std::string err;
};

namespace {

constexpr double CS2 = 1.0 / 3.0;

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

int validate(const lbm_params* p, lbm_derived* d) {
  if (!p) return LBM_EINVAL;
  if (p->nx < 1 || p->ny < 1) return LBM_EINVAL;
  if (p->bc_x < 0 || p->bc_x > 1 || p->bc_y < 0 || p->bc_y > 1) return LBM_EINVAL;
  if (p->precision != 32 && p->precision != 64) return LBM_EINVAL;
  if (p->diag_every < 0) return LBM_EINVAL;
  const size_t pitch = round_up((size_t)p->nx, 64);
  if (pitch * (size_t)p->ny > (size_t)INT32_MAX) return LBM_EINVAL;
  const double dphi = p->phi_A - p->phi_B;
  if (!(dphi != 0.0) || !std::isfinite(dphi)) return LBM_EINVAL;
  if (!(p->rho_A > 0) || !(p->rho_B > 0) || !(p->nu_A > 0) || !(p->nu_B > 0)) return LBM_EINVAL;
  if (!(p->M > 0) || !(p->alpha > 0)) return LBM_EINVAL;
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
  r.alpha = p->alpha;
  r.tau_f = 0.5 + p->M / (CS2 * p->alpha);
  r.tau_gA = 0.5 + p->nu_A / CS2;
  r.tau_gB = 0.5 + p->nu_B / CS2;
  if (!(r.tau_f > 0.5) || !(r.tau_gA > 0.5) || !(r.tau_gB > 0.5)) return LBM_EINVAL;
  if (d) *d = r;
  return LBM_OK;
}

struct Layout {
  size_t pitch, ps, esz;
  size_t state_bytes, ws_bytes;
  int ntx1, nty1, ntx2, nty2;
};

Layout layout_of(const lbm_params* p) {
  Layout L;
  L.esz = p->precision == 32 ? 4 : 8;
  L.pitch = round_up((size_t)p->nx, 64);
  // Plane stride: 256-byte multiple plus 4 KiB of padding so that the 18
  // planes read together do not sit at addresses a power of two apart.
  L.ps = round_up(L.pitch * (size_t)p->ny, 256 / L.esz) + 4096 / L.esz;
  L.state_bytes = (2 * NPOP + 3) * L.ps * L.esz;
  L.ntx1 = (p->nx + K1_TX - 1) / K1_TX;
  L.nty1 = (p->ny + K1_TY - 1) / K1_TY;
  L.ntx2 = (p->nx + K2_TX - 1) / K2_TX;
  L.nty2 = (p->ny + K2_TY - 1) / K2_TY;
  const size_t nparts = (size_t)L.ntx2 * L.nty2;
  L.ws_bytes = round_up((nparts * NQ + 2 * NQ) * sizeof(double), 256);
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
  return plane<T>(c, which * NPOP);
}
template <typename T>
T* S_plane(lbm_ctx* c) { return plane<T>(c, 2 * NPOP); }
template <typename T>
T* dphi_plane(lbm_ctx* c) { return plane<T>(c, 2 * NPOP + 1); }
template <typename T>
T* mu_plane(lbm_ctx* c) { return plane<T>(c, 2 * NPOP + 2); }

unsigned blocks_for(long long n) { return (unsigned)((n + 255) / 256); }

template <typename T>
int launch_phi_mu(lbm_ctx* c) {
  hipLaunchKernelGGL((k_phi_mu<T, false>), dim3(c->ntx1 * c->nty1), dim3(256), 0, c->stream, c->kp,
                     popbuf<T>(c, c->cur), nullptr, dphi_plane<T>(c), mu_plane<T>(c), c->ntx1);
  LAUNCHCHK(c);
  return LBM_OK;
}

template <typename T, int MODE>
int launch_collide(lbm_ctx* c, MomOut mo) {
  hipLaunchKernelGGL((k_collide<T, MODE>), dim3(c->ntx2 * c->nty2), dim3(256), 0, c->stream, c->kp,
                     popbuf<T>(c, c->cur), popbuf<T>(c, c->cur ^ 1), S_plane<T>(c), dphi_plane<T>(c),
                     mu_plane<T>(c), mo, c->partials, c->ntx2);
  LAUNCHCHK(c);
  return LBM_OK;
}

int launch_reduce(lbm_ctx* c, int slot) {
  hipLaunchKernelGGL(k_reduce_diag, dim3(1), dim3(256), 0, c->stream, c->partials,
                     c->ntx2 * c->nty2, c->diag_dev + slot * NQ);
  LAUNCHCHK(c);
  return LBM_OK;
}

void fill_diag(const double* v, int64_t step, lbm_diag* d) {
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

template <typename T>
int step_impl(lbm_ctx* c, int64_t n) {
  for (int64_t k = 0; k < n; ++k) {
    const bool diag = c->p.diag_every > 0 && (c->step % c->p.diag_every) == 0;
    if (c->timing) {
      hipEvent_t e[3];
      for (int j = 0; j < 3; ++j) {
        HIPCHK(c, hipEventCreate(&e[j]));
        c->tev.push_back(e[j]);
      }
      HIPCHK(c, hipEventRecord(e[0], c->stream));
      int r = launch_phi_mu<T>(c);
      if (r) return r;
      HIPCHK(c, hipEventRecord(e[1], c->stream));
      r = diag ? launch_collide<T, M_STEP_DIAG>(c, MomOut{}) : launch_collide<T, M_STEP>(c, MomOut{});
      if (r) return r;
      HIPCHK(c, hipEventRecord(e[2], c->stream));
    } else {
      int r = launch_phi_mu<T>(c);
      if (r) return r;
      r = diag ? launch_collide<T, M_STEP_DIAG>(c, MomOut{}) : launch_collide<T, M_STEP>(c, MomOut{});
      if (r) return r;
    }
    if (diag) {
      int r = consume_diag(c, true);  // the host buffer is about to be reused
      if (r) return r;
      r = launch_reduce(c, 0);
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
  hipLaunchKernelGGL(k_init_pops<T>, dim3(blocks_for(n)), dim3(256), 0, c->stream, c->kp,
                     popbuf<T>(c, c->cur), phi0, ux0, uy0, mu_plane<T>(c));
  LAUNCHCHK(c);
  int r = launch_phi_mu<T>(c);
  if (r) return r;
  return launch_collide<T, M_INIT_S>(c, MomOut{});
}

template <typename T>
int moments_impl(lbm_ctx* c, MomOut mo, lbm_diag* diag) {
  int r = launch_phi_mu<T>(c);
  if (r) return r;
  r = launch_collide<T, M_MOMENTS>(c, mo);
  if (r) return r;
  if (diag) {
    r = launch_reduce(c, 1);
    if (r) return r;
    HIPCHK(c, hipMemcpyAsync(c->diag_host + NQ, c->diag_dev + NQ, NQ * sizeof(double),
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    fill_diag(c->diag_host + NQ, c->step, diag);
  }
  return LBM_OK;
}

template <typename T>
int get_state_impl(lbm_ctx* c, int x0, int y0, int w, int h, double* f, double* g, double* Sp) {
  const long long n = (long long)w * h;
  hipLaunchKernelGGL(k_get_state<T>, dim3(blocks_for(n)), dim3(256), 0, c->stream, c->kp,
                     popbuf<T>(c, c->cur), S_plane<T>(c), x0, y0, w, h, f, g, Sp);
  LAUNCHCHK(c);
  return LBM_OK;
}

template <typename T>
int set_state_impl(lbm_ctx* c, const double* f, const double* g, const double* Sp) {
  const long long n = (long long)c->p.nx * c->p.ny;
  hipLaunchKernelGGL(k_set_state<T>, dim3(blocks_for(n)), dim3(256), 0, c->stream, c->kp,
                     popbuf<T>(c, c->cur), S_plane<T>(c), f, g, Sp);
  LAUNCHCHK(c);
  return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_derive(const lbm_params* p, lbm_derived* out) { return validate(p, out); }

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
  lbm_ctx* c = new lbm_ctx();
  c->p = *p;
  c->d = d;
  const Layout L = layout_of(p);
  c->prec = p->precision;
  c->esz = L.esz;
  c->state = static_cast<char*>(state);
  c->ws = static_cast<char*>(workspace);
  c->stream = static_cast<hipStream_t>(stream);
  c->cur = 0;
  c->step = 0;
  c->ntx1 = L.ntx1;
  c->nty1 = L.nty1;
  c->ntx2 = L.ntx2;
  c->nty2 = L.nty2;
  c->partials = reinterpret_cast<double*>(c->ws);
  c->diag_dev = c->partials + (size_t)L.ntx2 * L.nty2 * NQ;
  c->diag_pending = c->diag_seen = c->nonfinite = false;
  c->timing = false;
  KP& k = c->kp;
  k.nx = p->nx;
  k.ny = p->ny;
  k.pitch = (int)L.pitch;
  k.bcx = p->bc_x;
  k.bcy = p->bc_y;
  k.ps = (long long)L.ps;
  const double dphi = p->phi_A - p->phi_B;
  k.phi_ref = p->precision == 32 ? 0.5 * (p->phi_A + p->phi_B) : 0.0;
  k.cA = k.phi_ref - p->phi_A;
  k.cB = k.phi_ref - p->phi_B;
  k.beta4 = 4.0 * d.beta;
  k.kappa = d.kappa;
  k.alpha = p->alpha;
  k.omega_f = 1.0 / d.tau_f;
  k.rhoB = p->rho_B;
  k.drho = (p->rho_A - p->rho_B) / dphi;
  k.tgB = d.tau_gB;
  k.dtg = (d.tau_gA - d.tau_gB) / dphi;
  k.gx = p->gx;
  k.gy = p->gy;
  hipError_t e = hipHostMalloc((void**)&c->diag_host, 2 * NQ * sizeof(double), hipHostMallocDefault);
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
  fill_diag(c->diag_host, c->diag_step, diag);
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
  c->timing = enable != 0;
  return LBM_OK;
}

int lbm_kernel_times(lbm_ctx* c, double* ms_phi_mu, double* ms_collide, int64_t* steps) {
  if (!c) return LBM_EINVAL;
  HIPCHK(c, hipStreamSynchronize(c->stream));
  double a = 0.0, b = 0.0;
  for (size_t k = 0; k + 2 < c->tev.size(); k += 3) {
    float t1 = 0.f, t2 = 0.f;
    HIPCHK(c, hipEventElapsedTime(&t1, c->tev[k], c->tev[k + 1]));
    HIPCHK(c, hipEventElapsedTime(&t2, c->tev[k + 1], c->tev[k + 2]));
    a += t1;
    b += t2;
  }
  if (ms_phi_mu) *ms_phi_mu = a;
  if (ms_collide) *ms_collide = b;
  if (steps) *steps = (int64_t)(c->tev.size() / 3);
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
