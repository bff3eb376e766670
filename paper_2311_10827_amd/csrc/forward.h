// Forward kernels of one time step of the well-balanced phase-field LBM
// (Ju et al., arXiv 2311.10827): the step as one kernel (k_step_fused: phi,
// mu and the collide-and-pull-stream of a marching strip, phi and mu kept in
// LDS) or as two (k_phi_mu, the phi/mu stencil pass K1, then k_collide, the
// collide-and-pull-stream pass K2), plus initialisation and state I/O.
//
// FP64 arithmetic is written term by term in the order of the plain
// definitions (sums over the velocity set in index order, no fused
// multiply-add: the library is compiled with -ffp-contract=off), so the FP64
// step is reproducible against any implementation of the same definitions in
// that order.  The FP32 path uses difference forms that keep small
// quantities small: stencils as differences phi(x + c) - phi(x), factored
// double-well, and the f_0 update as an increment added to hi + lo.
#pragma once
#include "common.h"

namespace lbm {

// ---------------------------------------------------------- FP64 operators
// Isotropic gradient (Sec. 2.3.2, eq. gradient),
//   grad Psi = sum_{i=1..8} w_i c_i Psi(x + c_i) / c_s^2,
// accumulated over i = 1..8 in index order (terms with c_i = 0 omitted).
// v[dy+1][dx+1] holds Psi(x + dx, y + dy).
__device__ __forceinline__ void grad_f64(const double (&v)[3][3], double& gx, double& gy) {
  const double w1 = w_of(1), w5 = w_of(5);
  double ax = (w1 * v[1][2]) * INV_CS2;     // 1 E
  ax = ax + ((-w1) * v[1][0]) * INV_CS2;    // 3 W
  ax = ax + (w5 * v[2][2]) * INV_CS2;       // 5 NE
  ax = ax + ((-w5) * v[2][0]) * INV_CS2;    // 6 NW
  ax = ax + ((-w5) * v[0][0]) * INV_CS2;    // 7 SW
  ax = ax + (w5 * v[0][2]) * INV_CS2;       // 8 SE
  double ay = (w1 * v[2][1]) * INV_CS2;     // 2 N
  ay = ay + ((-w1) * v[0][1]) * INV_CS2;    // 4 S
  ay = ay + (w5 * v[2][2]) * INV_CS2;       // 5 NE
  ay = ay + (w5 * v[2][0]) * INV_CS2;       // 6 NW
  ay = ay + ((-w5) * v[0][0]) * INV_CS2;    // 7 SW
  ay = ay + ((-w5) * v[0][2]) * INV_CS2;    // 8 SE
  gx = ax;
  gy = ay;
}

// Isotropic Laplacian (Sec. 2.3.2, eq. Laplace),
//   lap Psi = sum_{i=1..8} 2 w_i [Psi(x + c_i) - Psi(x)] / c_s^2, i in index order.
__device__ __forceinline__ double lap_f64(const double (&v)[3][3]) {
  const double a1 = 2.0 * w_of(1), a5 = 2.0 * w_of(5);
  const double c = v[1][1];
  double a = (a1 * (v[1][2] - c)) * INV_CS2;  // E
  a = a + (a1 * (v[2][1] - c)) * INV_CS2;     // N
  a = a + (a1 * (v[1][0] - c)) * INV_CS2;     // W
  a = a + (a1 * (v[0][1] - c)) * INV_CS2;     // S
  a = a + (a5 * (v[2][2] - c)) * INV_CS2;     // NE
  a = a + (a5 * (v[2][0] - c)) * INV_CS2;     // NW
  a = a + (a5 * (v[0][0] - c)) * INV_CS2;     // SW
  a = a + (a5 * (v[0][2] - c)) * INV_CS2;     // SE
  return a;
}

// s_i(u) of Sec. 2.3.2, eq. Siu:
//   w_i [c.u / c_s^2 + (c.u)^2 / (2 c_s^4) - u.u / (2 c_s^2)].
__device__ __forceinline__ double s_f64(int i, double ux, double uy, double uu) {
  const double cu = (double)cx_of(i) * ux + (double)cy_of(i) * uy;
  return w_of(i) * ((cu * INV_CS2 + ((0.5 * cu) * cu) * INV_CS2 * INV_CS2) - (0.5 * uu) * INV_CS2);
}

// phi - phi_ref of a cell from its gathered f (Sec. 2.3.1, eq. order-parameter):
// FP64 sums f_0..f_8 in index order; FP32 adds the small sum to hi + lo.
template <typename T>
__device__ __forceinline__ T phi_sum(const Pops<T>& q) {
  if constexpr (std::is_same<T, double>::value) {
    double a = q.f[0];
#pragma unroll
    for (int i = 1; i < 9; ++i) a = a + q.f[i];
    return a;
  } else {
    const float s8 = ((q.f[1] + q.f[2]) + (q.f[3] + q.f[4])) + ((q.f[5] + q.f[6]) + (q.f[7] + q.f[8]));
    return q.f[0] + (q.lo + s8);
  }
}

// mu = 4 beta (phi - phi_A)(phi - phi_B)(phi - phi_m) - kappa lap(phi)
// (Sec. 2.1, eq. chemical_potencial; Sec. 2.3.2, eq. Laplace) from the 3x3
// values of phi - phi_ref, v[dy+1][dx+1].  FP64 in plain-definition order;
// FP32 in difference form.
template <typename C>
__device__ __forceinline__ C mu_cell(const KP& p, const C (&v)[3][3]) {
  const C c = v[1][1];
  if constexpr (std::is_same<C, double>::value) {
    const double ph = c + p.phi_ref;
    const double lap = lap_f64(v);
    return (((p.beta4 * (ph - p.phiA)) * (ph - p.phiB)) * (ph - p.phim)) - p.kappa * lap;
  } else {
    // FP32: a * b + c may fuse (each such expression as written, so every
    // FP32 kernel gets the same bits)
#pragma clang fp contract(on)
    const C axis = ((v[1][2] - c) + (v[1][0] - c)) + ((v[2][1] - c) + (v[0][1] - c));
    const C diag = ((v[2][2] - c) + (v[2][0] - c)) + ((v[0][2] - c) + (v[0][0] - c));
    const C lap = (C)(2.0 / 3.0) * axis + (C)(1.0 / 6.0) * diag;
    const C dA = c + (C)(p.phi_ref - p.phiA), dB = c + (C)(p.phi_ref - p.phiB);
    const C dm = c + (C)(p.phi_ref - p.phim);
    return ((C)p.beta4 * (dA * dB)) * dm - (C)p.kappa * lap;
  }
}

// ----------------------------------------------------------- K1: phi and mu
// phi = sum_i f_i (Sec. 2.3.1, eq. order-parameter) on a tile plus a one-cell
// ring, staged in LDS; then mu = 4 beta (phi - phi_A)(phi - phi_B)(phi - phi_m)
// - kappa lap(phi) (Sec. 2.1, eq. chemical_potencial).  The dphi plane gets
// phi - phi_ref.  FROM_INPUT: phi comes from the caller's FP64 field
// (initialisation); then the arithmetic is FP64 whatever the storage type.
constexpr int K1_TX = 64, K1_TY = 16;

template <typename T, bool FROM_INPUT, bool LO16 = false>
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
      Pops<T> q;
      gather<false, T, true, true, LO16>(B, p, gx, gy, q);
      v = (C)phi_sum<T>(q);
    }
    s[k] = v;
  }
  __syncthreads();
  const int lx = threadIdx.x % K1_TX;
  for (int ly = threadIdx.x / K1_TX; ly < K1_TY; ly += blockDim.x / K1_TX) {
    const int x = x0 + lx, y = y0 + ly;
    if (x >= p.nx || y >= p.ny) continue;
    const C* r0 = s + ly * LW + lx;  // row y-1 starting at column x-1
    const C* r1 = r0 + LW;
    const C* r2 = r1 + LW;
    const C v[3][3] = {{r0[0], r0[1], r0[2]}, {r1[0], r1[1], r1[2]}, {r2[0], r2[1], r2[2]}};
    const long long o = (long long)y * p.pitch + x;
    dphi_out[o] = (T)v[1][1];
    mu_out[o] = (T)mu_cell<C>(p, v);
  }
}

// ---------------------------------------------------- K2: collide + stream
// Per cell: gather f_i, g_i (pull streaming with bounce-back), read the 3x3
// neighbourhoods of phi and mu, and apply
//   grad phi, grad mu, grad rho (Sec. 2.3.2, eq. gradient);
//   rho linear in phi, nu linear (Sec. 2.3.2, eq. vis) or in one of the two
//     alternative forms named there, tau_g = 1/2 + nu / c_s^2;
//   F = -phi grad mu + G (Sec. 2.1 after eq. 6; Sec. 2.3.2 after eq. GGi);
//   rho u = sum c_i g_i + F/2, p = c_s^2/(1-w_0)[sum_{i!=0} g_i + u.grad(rho)/2
//     + rho s_0(u)] (Sec. 2.3.2, macroscopic subequations);
//   S = u.grad phi; the f collision with F_i(S) + [F_i(S) - F_i(S_prev)]/2
//     (Sec. 2.3.1, eqs. BGK, H_i, F_i; backward difference in time);
//   the g collision with g^eq and G_i (Sec. 2.3.2, eqs. BGK-NS, G_i, Siu, GGi).
// The result is written at the cell itself into the other buffer (the next
// step's pull gather does the streaming); S replaces S_prev in place.
enum Mode { M_STEP = 0, M_STEP_DIAG = 1, M_MOMENTS = 2, M_INIT_S = 3 };

struct MomOut {
  double *phi, *mu, *ux, *uy, *p, *rho;
};

constexpr int K2_TX = 64, K2_TY = 4;

template <typename T>
struct Nbhd {
  T ph[3][3], mu[3][3];  // [dy+1][dx+1]
};

template <typename T>
__device__ __forceinline__ void load_nbhd(const KP& p, const T* __restrict__ dphi,
                                          const T* __restrict__ mupl, int x, int y, Nbhd<T>& n) {
  const int xs[3] = {stencil_idx(x - 1, p.nx, p.bcx), x, stencil_idx(x + 1, p.nx, p.bcx)};
  const int ys[3] = {stencil_idx(y - 1, p.ny, p.bcy), y, stencil_idx(y + 1, p.ny, p.bcy)};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const unsigned r = (unsigned)(ys[a] * p.pitch);
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      n.ph[a][b] = dphi[r + (unsigned)xs[b]];
      n.mu[a][b] = mupl[r + (unsigned)xs[b]];
    }
  }
}

// Macroscopic quantities of one cell, in FP64 (for moments and diagnostics).
struct CellOut {
  double phi, mu, ux, uy, p, rho, S, Sp;
};

// FP64 cell update, plain-definition order.  Writes the post-collision
// populations to fo/go when WRITE is set; MRT selects the moment-space
// collision in place of BGK.
template <bool WRITE, bool MRT = false>
__device__ __forceinline__ void cell_f64(const KP& p, const Pops<double>& q, const Nbhd<double>& n,
                                         double Sp, double (&fo)[9], double (&go)[9], CellOut& out) {
  double rho3[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) rho3[a][b] = p.rhoB + (n.ph[a][b] - p.phiB) * p.rho_slope;
  const double phi = n.ph[1][1], mu = n.mu[1][1], rho = rho3[1][1];
  const double nu = visc<double>(p, phi - p.phiB);
  double gpx, gpy, gmx, gmy, grx, gry;
  grad_f64(n.ph, gpx, gpy);
  grad_f64(n.mu, gmx, gmy);
  grad_f64(rho3, grx, gry);
  const double Fx = (-phi) * gmx + p.gx;
  const double Fy = (-phi) * gmy + p.gy;
  const double* g = q.g;
  const double mx = ((((g[1] - g[3]) + g[5]) - g[6]) - g[7]) + g[8];
  const double my = ((((g[2] - g[4]) + g[5]) + g[6]) - g[7]) - g[8];
  double snz = g[1];
#pragma unroll
  for (int i = 2; i < 9; ++i) snz = snz + g[i];
  const double ux = (mx + 0.5 * Fx) / rho;
  const double uy = (my + 0.5 * Fy) / rho;
  const double uu = ux * ux + uy * uy;
  const double s0 = w_of(0) * (0.0 - (0.5 * uu) * INV_CS2);
  const double pr = (CS2 / (1.0 - w_of(0))) * ((snz + 0.5 * (ux * grx + uy * gry)) + rho * s0);
  const double S = ux * gpx + uy * gpy;
  out = CellOut{phi, mu, ux, uy, pr, rho, S, Sp};
  if (!WRITE) return;
  // order-parameter population (Sec. 2.3.1, eqs. BGK, H_i, F_i)
  const double* f = q.f;
  double dfe[9];  // MRT: f^eq - f
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const double feq = i == 0 ? phi - ((1.0 - w_of(0)) * p.alpha) * mu : (w_of(i) * p.alpha) * mu;
    const double Fn = (w_of(i) * S) * src_bracket(i);
    const double Fo = (w_of(i) * Sp) * src_bracket(i);
    fo[i] = ((f[i] - p.omega_f * (f[i] - feq)) + Fn) + 0.5 * (Fn - Fo);
    if constexpr (MRT) dfe[i] = feq - f[i];
  }
  if constexpr (MRT) {  // the BGK update above plus the MRT correction
    double corr[9];
    mrt_corr_f(p, p.omega_f, dfe, corr);
#pragma unroll
    for (int i = 0; i < 9; ++i) fo[i] += corr[i];
  }
  // hydrodynamic population (Sec. 2.3.2, eqs. BGK-NS, G_i, Siu, GGi)
  const double tau = 0.5 + nu * INV_CS2;
  const double wg = 1.0 / tau;
  const double kG = 1.0 - 1.0 / (2.0 * tau);
  const double ugr = ux * grx + uy * gry;
  double z[9];  // MRT: (g^eq - g) - G~/2
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const double cx = cx_of(i), cy = cy_of(i);
    const double geq = (i == 0 ? (pr * INV_CS2) * (w_of(0) - 1.0) : (pr * INV_CS2) * w_of(i)) +
                       rho * s_f64(i, ux, uy, uu);
    const double cF = cx * Fx + cy * Fy;
    const double a = (double)(cx_of(i) * cx_of(i)) - CS2;
    const double b = (double)(cx_of(i) * cy_of(i));
    const double d = (double)(cy_of(i) * cy_of(i)) - CS2;
    const double dyad = (((ux * grx) * a + (ux * gry) * b) + (uy * grx) * b) + (uy * gry) * d;
    const double Gi = (kG * w_of(i)) * ((ugr + cF * INV_CS2) + dyad * INV_CS2);
    go[i] = (g[i] - wg * (g[i] - geq)) + Gi;
    if constexpr (MRT) z[i] = (geq - g[i]) - 0.5 * (w_of(i) * ((ugr + cF * INV_CS2) + dyad * INV_CS2));
  }
  if constexpr (MRT) {
    double corr[9];
    mrt_corr_g(p, wg, z, corr);
#pragma unroll
    for (int i = 0; i < 9; ++i) go[i] += corr[i];
  }
}

// FP32 cell update in difference forms.  fo[0] receives hi, fo_lo the low word.
template <bool WRITE, bool MRT = false>
__device__ __forceinline__ void cell_f32(const KP& p, const Pops<float>& q, const Nbhd<float>& n,
                                         float Sp, float (&fo)[9], float& fo_lo, float (&go)[9],
                                         CellOut& out) {
  // a * b + c may fuse (each such expression as written, so every FP32
  // kernel gets the same bits); the TwoSum of f_0 has no products
#pragma clang fp contract(on)
  const float third = (float)(1.0 / 3.0), twelfth = (float)(1.0 / 12.0);
  const auto& ph = n.ph;
  const auto& m = n.mu;
  const float gpx = third * (ph[1][2] - ph[1][0]) + twelfth * ((ph[2][2] - ph[2][0]) + (ph[0][2] - ph[0][0]));
  const float gpy = third * (ph[2][1] - ph[0][1]) + twelfth * ((ph[2][2] - ph[0][2]) + (ph[2][0] - ph[0][0]));
  const float gmx = third * (m[1][2] - m[1][0]) + twelfth * ((m[2][2] - m[2][0]) + (m[0][2] - m[0][0]));
  const float gmy = third * (m[2][1] - m[0][1]) + twelfth * ((m[2][2] - m[0][2]) + (m[2][0] - m[0][0]));
  const float dph = ph[1][1];  // phi - phi_ref
  const float phi = dph + (float)p.phi_ref;
  const float mu = m[1][1];
  const float dB = dph + (float)(p.phi_ref - p.phiB);
  const float drho = (float)p.rho_slope;
  const float rho = (float)p.rhoB + dB * drho;
  const float grx = drho * gpx, gry = drho * gpy;
  const float Fx = (float)p.gx - phi * gmx, Fy = (float)p.gy - phi * gmy;
  const float* g = q.g;
  const float mx = ((g[1] - g[3]) + (g[5] - g[7])) + (g[8] - g[6]);
  const float my = ((g[2] - g[4]) + (g[5] - g[7])) + (g[6] - g[8]);
  const float gnz = ((g[1] + g[2]) + (g[3] + g[4])) + ((g[5] + g[6]) + (g[7] + g[8]));
  const float irho = recip(rho);  // the hardware reciprocal (1 ulp)
  const float ux = (mx + 0.5f * Fx) * irho, uy = (my + 0.5f * Fy) * irho;
  const float uu = ux * ux + uy * uy;
  const float ugr = ux * grx + uy * gry;
  const float pr = 0.6f * (gnz + 0.5f * ugr - (float)(2.0 / 3.0) * rho * uu);
  const float S = ux * gpx + uy * gpy;
  const float* f = q.f;
  const float s8 = ((f[1] + f[2]) + (f[3] + f[4])) + ((f[5] + f[6]) + (f[7] + f[8]));
  out.phi = p.phi_ref + ((double)f[0] + ((double)q.lo + (double)s8));
  out.mu = mu;
  out.ux = ux;
  out.uy = uy;
  out.p = pr;
  out.rho = rho;
  out.S = S;
  out.Sp = Sp;
  if (!WRITE) return;
  const float src = 1.5f * S - 0.5f * Sp;
  const float wf = (float)p.omega_f;
  const float am = (float)p.alpha * mu;
  // f_0 - f_0^eq = -(s8 - (5/9) alpha mu) exactly, since phi = f_0 + s8; add the
  // small increment to hi + lo (TwoSum keeps the rounding error in lo, which
  // then never exceeds half an ulp of hi).
  float corr_f[9];  // MRT: the correction to the BGK update
  if constexpr (MRT) {
    // f^eq_0 - f_0 = s8 - (5/9) alpha mu exactly (phi = f_0 + s8)
    float d[9];
    d[0] = s8 - (float)(5.0 / 9.0) * am;
#pragma unroll
    for (int i = 1; i < 9; ++i) d[i] = (float)w_of(i) * am - f[i];
    mrt_corr_f(p, wf, d, corr_f);
  }
  float inc0 = wf * (s8 - (float)(5.0 / 9.0) * am) + (float)(w_of(0) * src_bracket(0)) * src;
  if constexpr (MRT) inc0 += corr_f[0];
  const float t = q.lo + inc0;
  const float hi = f[0] + t;
  const float tv = hi - f[0];
  fo[0] = hi;
  fo_lo = (f[0] - (hi - tv)) + (t - tv);
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    fo[i] = f[i] + wf * ((float)w_of(i) * am - f[i]) + (float)(w_of(i) * src_bracket(i)) * src;
    if constexpr (MRT) fo[i] += corr_f[i];
  }
  const float tau = 0.5f + 3.0f * visc<float>(p, dB);
  const float wg = recip(tau);
  const float kG = 1.0f - 0.5f * wg;
  const float ge0 = -(float)(5.0 / 3.0) * pr - (float)(2.0 / 3.0) * rho * uu;
  go[0] = g[0] + wg * (ge0 - g[0]);
  float z[9];  // MRT: (g^eq - g) - G~/2
  if constexpr (MRT) z[0] = ge0 - g[0];  // G~_0 vanishes: its u.grad(rho) terms cancel
  const float p3 = 3.0f * pr, ruu = 1.5f * rho * uu;
  // Directions in opposite pairs (i, opp(i)), c_opp = -c_i: with s the part
  // of g^eq_i and of the forcing G~_i even in c_i and a the odd part,
  //   g^eq = w (3p - 1.5 rho u.u + 4.5 rho (c.u)^2) + w 3 rho (c.u),
  //   G~   = 3 kG w (c.u)(c.grad rho) + 3 kG w (c.F),
  // and g_out = g + wg (g^eq - g) + G~ = (1 - wg) g + (wg s_eq + s_G) +- (wg a_eq + a_G).
  const float keep = 1.0f - wg;
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    if (i != 1 && i != 2 && i != 5 && i != 6) continue;  // i: 1 E, 2 N, 5 NE, 6 NW; opp 3, 4, 7, 8
    const int j = opp_of(i);
    const float cu = (float)cx_of(i) * ux + (float)cy_of(i) * uy;
    const float cF = (float)cx_of(i) * Fx + (float)cy_of(i) * Fy;
    const float cr = (float)cx_of(i) * grx + (float)cy_of(i) * gry;
    const float w = (float)w_of(i);
    const float s_eq = w * (p3 - ruu + 4.5f * rho * (cu * cu)), a_eq = (3.0f * w) * (rho * cu);
    const float s_G = (3.0f * w) * kG * (cu * cr), a_G = (3.0f * w) * kG * cF;
    const float A = wg * s_eq + s_G, B = wg * a_eq + a_G;
    go[i] = keep * g[i] + A + B;
    go[j] = keep * g[j] + A - B;
    if constexpr (MRT) {
      const float s_z = s_eq - (1.5f * w) * (cu * cr), a_z = a_eq - (1.5f * w) * cF;
      z[i] = (s_z + a_z) - g[i];
      z[j] = (s_z - a_z) - g[j];
    }
  }
  if constexpr (MRT) {
    float corr[9];
    mrt_corr_g(p, wg, z, corr);
#pragma unroll
    for (int i = 0; i < 9; ++i) go[i] += corr[i];
  }
}

// Spin holds S_prev of the current step; Spout receives S (they may be the
// same plane: each cell reads and then writes only its own entry).
template <typename T, int MODE, bool MRT = false, bool LO16 = false>
__global__ __launch_bounds__(256) void k_collide(const KP p, const T* Bin, T* Bout, const T* Spin,
                                                  T* Spout, const T* __restrict__ dphi,
                                                  const T* __restrict__ mupl, MomOut mo,
                                                  double* __restrict__ partials, int ntx) {
  constexpr bool DIAG = MODE == M_STEP_DIAG || MODE == M_MOMENTS;
  constexpr bool WRITE = MODE == M_STEP || MODE == M_STEP_DIAG;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int x = (tile % ntx) * K2_TX + (threadIdx.x & (K2_TX - 1));
  const int y = (tile / ntx) * K2_TY + threadIdx.x / K2_TX;
  const bool valid = x < p.nx && y < p.ny;
  Diag dg;
  if (DIAG) diag_identity(dg);
  if (valid) {
    const unsigned o = (unsigned)(y * p.pitch + x);
    Pops<T> q;
    gather<true, T, true, true, LO16>(Bin, p, x, y, q);
    Nbhd<T> nb;
    load_nbhd(p, dphi, mupl, x, y, nb);
    const T Sp = Spin[o];
    T fo[9], go[9];
    T lo = 0;
    CellOut c;
    if constexpr (std::is_same<T, double>::value)
      cell_f64<WRITE, MRT>(p, q, nb, Sp, fo, go, c);
    else
      cell_f32<WRITE, MRT>(p, q, nb, Sp, fo, lo, go, c);
    if (WRITE) {
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        (Bout + i * p.ps)[o] = fo[i];
        (Bout + (9 + i) * p.ps)[o] = go[i];
      }
      if constexpr (std::is_same<T, float>::value) {
        if constexpr (LO16)
          lo_plane(Bout, p)[o] = lo_encode(fo[0], lo);
        else
          (Bout + LO_PLANE * p.ps)[o] = lo;
      }
      Spout[o] = (T)c.S;
    }
    if (MODE == M_INIT_S) Spout[o] = (T)c.S;
    if (MODE == M_MOMENTS) {
      const long long k = (long long)y * p.nx + x;
      if (mo.phi) mo.phi[k] = c.phi;
      if (mo.mu) mo.mu[k] = c.mu;
      if (mo.ux) mo.ux[k] = c.ux;
      if (mo.uy) mo.uy[k] = c.uy;
      if (mo.p) mo.p[k] = c.p;
      if (mo.rho) mo.rho[k] = c.rho;
    }
    if (DIAG) {
      const bool fin = isfinite(c.phi) && isfinite(c.mu) && isfinite(c.ux) && isfinite(c.uy) &&
                       isfinite(c.p);
      dg.v[0] = c.phi;
      dg.v[1] = 1.5 * c.S - 0.5 * c.Sp;
      dg.v[2] = 0.5 * c.rho * (c.ux * c.ux + c.uy * c.uy);
      dg.v[3] = sqrt(c.ux * c.ux + c.uy * c.uy);
      dg.v[4] = dg.v[5] = c.rho;
      dg.v[6] = dg.v[7] = c.mu;
      dg.v[8] = dg.v[9] = c.phi;
      dg.v[10] = fin ? 0.0 : 1.0;
    }
  }
  if (DIAG) block_reduce_write(dg, partials + (long long)tile * NQ);
}

// Two-level fixed-order reduction of n partials: block b of the first pass
// reduces the contiguous chunk [b*chunk, (b+1)*chunk) into out[b]; a single
// block then reduces those.  The assignment of partials to lanes depends
// only on n, so the result is bitwise reproducible.
constexpr int RED_BLOCKS = 1024;
// ------------------------------------------- fused step: phi, mu, collide
// One workgroup owns a strip of W columns and H rows and marches up it.
// Per row y it takes the f gathered at row y+2 to phi (5-row ring in LDS,
// W + 4 columns) and keeps the strip's own gathered f (FR-row ring),
// computes mu of row y+1 (3-row ring, W + 2 columns) and then collides row y
// with the same arithmetic as k_collide: f and the 3x3 phi and mu come from
// LDS, only g is gathered from memory.  Every population plane is read from
// HBM once (up to the ring recompute at strip edges); phi and mu never go to
// HBM unless WRITE_PHIMU asks for them (the adjoint's recompute keeps them).
// Same results as k_phi_mu + k_collide, bit for bit.
//
// The row loop is software-pipelined: the loads of the next row (f for phi
// of row y+3, g and S_prev of row y+1) are issued after row y's collision
// and before its stores.  Vector memory operations of a wave complete in
// issue order, so the wait for those loads at the top of the next iteration
// does not include this row's stores, and the loads are in flight across
// the stores, the ring updates and the barriers.
//
// Ghosts: ring entries outside the grid hold phi of the wrapped or mirrored
// cell; a mu entry just outside a wall holds mu of the adjacent cell (its
// stencil is shifted by one), which is what the two-kernel path reads
// through stencil_idx.
//
// Strip width W (= threads per workgroup) and the largest strip height H;
// the host lowers the height (a kernel argument) on small grids so that a
// launch has more workgroups.
template <typename T>
struct Strip;
// FR: rows in the LDS ring of the strip's gathered f.  Four rows (FP32, 40
// KiB) need no barrier beyond the two per row; three rows (FP64, 54 KiB, so
// that two workgroups fit a CU) need one more per row.
// H = 32: against 64-row strips, 1-2 % faster at 8192^2 and 16384^2 in both
// precisions on every allocation measured, although the f halo rows read
// per strip double; 16 and 24 rows are slower again, and much taller
// strips (up to one band of workgroups per column) slower still.
template <>
struct Strip<float> {
  static constexpr int W = 256, H = 32, FR = 4;
};
template <>
struct Strip<double> {
  static constexpr int W = 256, H = 32, FR = 3;
};

__device__ __forceinline__ int mod_pos(int a, int m) {
  const int r = a % m;
  return r < 0 ? r + m : r;
}

// A population store: streaming (non-temporal) when NT, else ordinary.
template <bool NT, typename T>
__device__ __forceinline__ void pop_store(T v, T* ptr) {
  if constexpr (NT)
    __builtin_nontemporal_store(v, ptr);
  else
    *ptr = v;
}

// NT: streaming population stores, for states larger than the last-level
// cache (nothing reads them before they leave it); ordinary stores when the
// state fits there, so that the next step finds them in it.  LO16: the FP32
// low word of f_0 in 16 bits.
template <typename T, int MODE, bool WRITE_PHIMU, bool MRT = false, bool NT = true, bool LO16 = false>
__global__ __launch_bounds__(Strip<T>::W) void k_step_fused(const KP p, const T* Bin, T* Bout, const T* Spin,
                                                             T* Spout, T* __restrict__ dphi_out,
                                                             T* __restrict__ mu_out,
                                                             double* __restrict__ partials, int ntx,
                                                             int H, int xcd_order) {
  constexpr bool DIAG = MODE == M_STEP_DIAG;
  constexpr int W = Strip<T>::W;
  constexpr int FR = Strip<T>::FR;
  static_assert(FR == 3 || FR == 4, "f ring of 3 or 4 rows");
  constexpr int NF = std::is_same<T, float>::value ? 10 : 9;  // f_0..f_8 (+ low word of f_0)
  __shared__ T phr[5][W + 4];     // phi - phi_ref, column x0 - 2 + k
  __shared__ T mur[3][W + 2];     // mu, column x0 - 1 + k
  __shared__ T fr[FR][NF][W];     // gathered f of the strip's own columns
  // strip order: XCD-contiguous bands, or the dispatch order itself (the
  // hardware deals consecutive workgroups to the eight XCDs in turn)
  const int blk = xcd_order ? xcd_tile(blockIdx.x, gridDim.x) : (int)blockIdx.x;
  const int x0 = (blk % ntx) * W, y0 = (blk / ntx) * H;
  const int y1 = y0 + H < p.ny ? y0 + H : p.ny;
  const int t = threadIdx.x;

  // f of the phi columns a thread owns in one row: k = t and, for t < 4,
  // k = W + t.
  struct PhiCols {
    Pops<T> a, b;
  };
  auto phi_load = [&](int yu, PhiCols& L) {
    const int gy = stencil_idx(yu, p.ny, p.bcy);
    gather<false, T, true, true, LO16>(Bin, p, stencil_idx(x0 - 2 + t, p.nx, p.bcx), gy, L.a);
    if (t < 4) gather<false, T, true, true, LO16>(Bin, p, stencil_idx(x0 - 2 + W + t, p.nx, p.bcx), gy, L.b);
  };
  // phi of row yu (unwrapped) into the ring; for rows this strip collides
  // the gathered f of its own columns is kept for the collision.
  auto phi_put = [&](int yu, const Pops<T>& q, int k) {
    const T v = phi_sum<T>(q);
    phr[mod_pos(yu, 5)][k] = v;
    if (yu >= y0 && yu < y1 && k >= 2 && k < W + 2) {
      T(*fk)[W] = fr[mod_pos(yu, FR)];
#pragma unroll
      for (int i = 0; i < 9; ++i) fk[i][k - 2] = q.f[i];
      if constexpr (NF == 10) fk[9][k - 2] = q.lo;
      if (WRITE_PHIMU && x0 - 2 + k < p.nx) dphi_out[(long long)yu * p.pitch + (x0 - 2 + k)] = v;
    }
  };
  auto phi_store = [&](int yu, const PhiCols& L) {
    phi_put(yu, L.a, t);
    if (t < 4) phi_put(yu, L.b, W + t);
  };
  auto mu_row = [&](int yu) {
    // stencil rows shifted inward for a ghost row beyond a wall
    const int sy = p.bcy ? (yu < 0 ? 1 : (yu >= p.ny ? -1 : 0)) : 0;
    const T* r0 = phr[mod_pos(yu + sy - 1, 5)];
    const T* r1 = phr[mod_pos(yu + sy, 5)];
    const T* r2 = phr[mod_pos(yu + sy + 1, 5)];
    T* out = mur[mod_pos(yu, 3)];
    for (int k = t; k < W + 2; k += W) {
      const int xu = x0 - 1 + k;
      const int sx = p.bcx ? (xu < 0 ? 1 : (xu >= p.nx ? -1 : 0)) : 0;
      const int c = k + 1 + sx;  // phi ring index of the stencil centre
      const T v[3][3] = {{r0[c - 1], r0[c], r0[c + 1]}, {r1[c - 1], r1[c], r1[c + 1]},
                         {r2[c - 1], r2[c], r2[c + 1]}};
      const T m = mu_cell<T>(p, v);
      out[k] = m;
      if (WRITE_PHIMU && yu >= y0 && yu < y1 && k >= 1 && k <= W && xu < p.nx)
        mu_out[(long long)yu * p.pitch + xu] = m;
    }
  };
  const int x = x0 + t;
  const bool active = x < p.nx;
  // g and S_prev of row y (its f is in the ring)
  auto row_load = [&](int y, Pops<T>& q, T& Sp) {
    gather<true, T, false>(Bin, p, x, y, q);
    Sp = Spin[(unsigned)(y * p.pitch + x)];
  };

  Diag dg;
  if (DIAG) diag_identity(dg);
  for (int r = y0 - 2; r <= y0 + 1; ++r) {
    PhiCols L;
    phi_load(r, L);
    phi_store(r, L);
  }
  __syncthreads();
  mu_row(y0 - 1);
  mu_row(y0);
  PhiCols L;
  Pops<T> q;
  T Sp = T(0);
  phi_load(y0 + 2, L);
  if (active) row_load(y0, q, Sp);
  // Ring hazards: phi_store(y+2) overwrites the phi slot of row y-3, read
  // last by mu_row(y-2) and the collision of row y-2, and the f slot of row
  // y-2 (FR = 4; the collision of row y-2 read it) or of row y-1 (FR = 3;
  // the collision of row y-1, hence the extra barrier); mu_row(y+1)
  // overwrites the slot of row y-2, read last by the collision of row y-1,
  // which finished before the first barrier of iteration y.
  for (int y = y0; y < y1; ++y) {
    if (FR == 3) __syncthreads();
    phi_store(y + 2, L);
    __syncthreads();
    mu_row(y + 1);
    __syncthreads();
    T fo[9], go[9];
    T lo = 0;
    CellOut c;
    if (active) {
      T(*fk)[W] = fr[mod_pos(y, FR)];
#pragma unroll
      for (int i = 0; i < 9; ++i) q.f[i] = fk[i][t];
      if constexpr (NF == 10) q.lo = fk[9][t];
      Nbhd<T> nb;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const T* pr = phr[mod_pos(y - 1 + a, 5)];
        const T* mr = mur[mod_pos(y - 1 + a, 3)];
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          nb.ph[a][b] = pr[t + 1 + b];
          nb.mu[a][b] = mr[t + b];
        }
      }
      if constexpr (std::is_same<T, double>::value)
        cell_f64<true, MRT>(p, q, nb, Sp, fo, go, c);
      else
        cell_f32<true, MRT>(p, q, nb, Sp, fo, lo, go, c);
    }
    // next row's loads go out before this row's stores
    if (y + 1 < y1) {
      phi_load(y + 3, L);
      if (active) row_load(y + 1, q, Sp);
    }
    if (active) {
      const unsigned o = (unsigned)(y * p.pitch + x);
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        pop_store<NT>(fo[i], Bout + i * p.ps + o);
        pop_store<NT>(go[i], Bout + (9 + i) * p.ps + o);
      }
      if constexpr (std::is_same<T, float>::value) {
        if constexpr (LO16)
          pop_store<NT>(lo_encode(fo[0], lo), lo_plane(Bout, p) + o);
        else
          pop_store<NT>(lo, Bout + LO_PLANE * p.ps + o);
      }
      pop_store<NT>((T)c.S, Spout + o);
      if (DIAG) {
        const bool fin = isfinite(c.phi) && isfinite(c.mu) && isfinite(c.ux) && isfinite(c.uy) &&
                         isfinite(c.p);
        Diag e;
        e.v[0] = c.phi;
        e.v[1] = 1.5 * c.S - 0.5 * c.Sp;
        e.v[2] = 0.5 * c.rho * (c.ux * c.ux + c.uy * c.uy);
        e.v[3] = sqrt(c.ux * c.ux + c.uy * c.uy);
        e.v[4] = e.v[5] = c.rho;
        e.v[6] = e.v[7] = c.mu;
        e.v[8] = e.v[9] = c.phi;
        e.v[10] = fin ? 0.0 : 1.0;
        for (int k = 0; k < NQ; ++k) dg.v[k] = diag_op(k, dg.v[k], e.v[k]);
      }
    }
  }
  if (DIAG) block_reduce_write(dg, partials + (long long)blk * NQ);
}

// Maximum of v over the 256 lanes of a block (every lane gets it).
__device__ __forceinline__ double block_max256(double v) {
  __shared__ double red[4];
  for (int s = 32; s >= 1; s >>= 1) v = fmax(v, __shfl_xor(v, s, 64));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  const double m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  __syncthreads();
  return m;
}

// max_x |div u| in FP64, first pass: div u = d_x u_x + d_y u_y, each
// derivative the isotropic gradient of Sec. 2.3.2 (eq. gradient), with the
// stencils' periodic wrap or mirrored wall ghosts, over dense velocity
// planes [ny][nx].  Block b takes cells b*256 + t, stepping by the whole
// grid, and writes its maximum to part[b]; non-finite values are left out
// (the non-finite count of the diagnostics reports them).
__global__ __launch_bounds__(256) void k_max_div_u(const KP p, const double* __restrict__ ux,
                                                    const double* __restrict__ uy,
                                                    double* __restrict__ part) {
  const long long n = (long long)p.nx * p.ny;
  double m = 0.0;
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x) {
    const int y = (int)(k / p.nx), x = (int)(k - (long long)y * p.nx);
    double dx = 0.0, dy = 0.0;
#pragma unroll
    for (int i = 1; i < 9; ++i) {
      const long long kn = (long long)stencil_idx(y + cy_of(i), p.ny, p.bcy) * p.nx +
                           stencil_idx(x + cx_of(i), p.nx, p.bcx);
      if (cx_of(i) != 0) dx = dx + ((w_of(i) * cx_of(i)) * ux[kn]) * INV_CS2;
      if (cy_of(i) != 0) dy = dy + ((w_of(i) * cy_of(i)) * uy[kn]) * INV_CS2;
    }
    const double d = fabs(dx + dy);
    if (isfinite(d)) m = fmax(m, d);
  }
  m = block_max256(m);
  if (threadIdx.x == 0) part[blockIdx.x] = m;
}

// Second pass: the maximum of n partials into out[0] (one block).  A
// maximum does not depend on the order it is taken in.
__global__ __launch_bounds__(256) void k_max_reduce(const double* __restrict__ part, int n,
                                                     double* __restrict__ out) {
  double m = 0.0;
  for (int k = threadIdx.x; k < n; k += blockDim.x) m = fmax(m, part[k]);
  m = block_max256(m);
  if (threadIdx.x == 0) out[0] = m;
}

// Sums of NV values over the 256 lanes of a block, in a fixed order (wave
// butterflies, then the four waves in order), written to out[0..NV) by
// thread 0.
template <int NV>
__device__ __forceinline__ void block_sum_write(double (&v)[NV], double* __restrict__ out) {
  __shared__ double red[4][NV];
#pragma unroll
  for (int k = 0; k < NV; ++k)
    for (int s = 32; s >= 1; s >>= 1) v[k] += __shfl_xor(v[k], s, 64);
  if ((threadIdx.x & 63) == 0)
    for (int k = 0; k < NV; ++k) red[threadIdx.x >> 6][k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
    for (int k = 0; k < NV; ++k) out[k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
}

// Laplace pressure jump, first pass.  P^ = p + phi mu - psi(phi), psi(phi) =
// beta (phi - phi_A)^2 (phi - phi_B)^2 (Sec. 2.1, eqs. bulk_energy,
// chemical_potencial), in FP64 from dense planes [ny][nx].  With the
// phase-A fraction s = (phi - phi_B) / (phi_A - phi_B), a cell is bulk A if
// s >= max(s) - LAP_BULK_TOL and bulk B if s <= min(s) + LAP_BULK_TOL; the
// extremes come from the grid's phi extrema (ext = {phi_min, phi_max}).
// Block b takes cells b*256 + t, stepping by the whole grid, and writes
// (sum of P^ over A, count A, sum over B, count B, count of cells in both)
// to part[5b..5b+5).
constexpr double LAP_BULK_TOL = 0.01;
__global__ __launch_bounds__(256) void k_laplace_part(const KP p, const double* __restrict__ phi,
                                                       const double* __restrict__ mu,
                                                       const double* __restrict__ pr,
                                                       const double* __restrict__ ext,
                                                       double* __restrict__ part) {
  const long long n = (long long)p.nx * p.ny;
  const double d = p.phiA - p.phiB, beta = 0.25 * p.beta4;
  const double s_lo = (ext[0] - p.phiB) / d, s_hi = (ext[1] - p.phiB) / d;
  const double a_min = fmax(s_lo, s_hi) - LAP_BULK_TOL, b_max = fmin(s_lo, s_hi) + LAP_BULK_TOL;
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x) {
    const double ph = phi[k];
    const double s = (ph - p.phiB) / d;
    const bool a = s >= a_min, b = s <= b_max;
    if (a || b) {
      const double dA = ph - p.phiA, dB = ph - p.phiB;
      const double hat = (pr[k] + ph * mu[k]) - (beta * (dA * dA)) * (dB * dB);
      if (a) {
        v[0] += hat;
        v[1] += 1.0;
      }
      if (b) {
        v[2] += hat;
        v[3] += 1.0;
      }
      if (a && b) v[4] += 1.0;
    }
  }
  block_sum_write<5>(v, part + 5 * (long long)blockIdx.x);
}

// Second pass: the n partial 5-tuples summed in a fixed order into out[0..5).
__global__ __launch_bounds__(256) void k_laplace_reduce(const double* __restrict__ part, int n,
                                                         double* __restrict__ out) {
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int k = threadIdx.x; k < n; k += blockDim.x)
    for (int j = 0; j < 5; ++j) v[j] += part[5 * k + j];
  block_sum_write<5>(v, out);
}

__global__ __launch_bounds__(256) void k_reduce_diag(const double* __restrict__ partials, long long n,
                                                      long long chunk, double* __restrict__ out) {
  Diag d;
  diag_identity(d);
  const long long b0 = (long long)blockIdx.x * chunk;
  const long long b1 = b0 + chunk < n ? b0 + chunk : n;
  for (long long b = b0 + threadIdx.x; b < b1; b += blockDim.x)
    for (int k = 0; k < NQ; ++k) d.v[k] = diag_op(k, d.v[k], partials[b * NQ + k]);
  block_reduce_write(d, out + (long long)blockIdx.x * NQ);
}

// ------------------------------------------------------------ state I/O
template <typename T, bool LO16>
__device__ __forceinline__ void put_f0(T* __restrict__ B, const KP& p, int x, int y, double v) {
  // the rest population never streams, so it is stored at the cell itself
  const long long own = (long long)y * p.pitch + x;
  if constexpr (std::is_same<T, float>::value) {
    float hi, lo;
    split2(v, hi, lo);
    B[own] = hi;
    if constexpr (LO16)
      lo_plane(B, p)[own] = lo_encode(hi, lo);
    else
      B[LO_PLANE * p.ps + own] = lo;
  } else {
    B[own] = v;
  }
}

// Initial populations (time 0): f = f^eq(phi0, mu0) (Sec. 2.3.1, eq. H_i) and
// g = g^eq(p = 0, u0) (Sec. 2.3.2, eqs. G_i, Siu), in FP64; mu0 comes from
// k_phi_mu<FROM_INPUT>.
template <typename T, bool LO16 = false>
__global__ __launch_bounds__(256) void k_init_pops(const KP p, T* __restrict__ B,
                                                    const double* __restrict__ phi0,
                                                    const double* __restrict__ ux0,
                                                    const double* __restrict__ uy0,
                                                    const T* __restrict__ mupl) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= (long long)p.nx * p.ny) return;
  const int y = (int)(k / p.nx), x = (int)(k - (long long)y * p.nx);
  const double ph = phi0[k];
  const double mu = (double)mupl[(long long)y * p.pitch + x];
  put_f0<T, LO16>(B, p, x, y, (ph - ((1.0 - w_of(0)) * p.alpha) * mu) - p.phi_ref);
  for (int i = 1; i < 9; ++i) scatter<T>(B, p, x, y, 0, i, (T)((w_of(i) * p.alpha) * mu));
  const double ux = ux0 ? ux0[k] : 0.0, uy = uy0 ? uy0[k] : 0.0;
  const double rho = p.rhoB + (ph - p.phiB) * p.rho_slope;
  const double uu = ux * ux + uy * uy;
  for (int i = 0; i < 9; ++i) scatter<T>(B, p, x, y, 9, i, (T)(rho * s_f64(i, ux, uy, uu)));
}

template <typename T, bool LO16 = false>
__global__ __launch_bounds__(256) void k_set_state(const KP p, T* __restrict__ B, T* __restrict__ Spl,
                                                    const double* __restrict__ f,
                                                    const double* __restrict__ g,
                                                    const double* __restrict__ Sp) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long n = (long long)p.nx * p.ny;
  if (k >= n) return;
  const int y = (int)(k / p.nx), x = (int)(k - (long long)y * p.nx);
  put_f0<T, LO16>(B, p, x, y, f[k] - p.phi_ref);
  for (int i = 1; i < 9; ++i) scatter<T>(B, p, x, y, 0, i, (T)f[i * n + k]);
  for (int i = 0; i < 9; ++i) scatter<T>(B, p, x, y, 9, i, (T)g[i * n + k]);
  Spl[(long long)y * p.pitch + x] = (T)Sp[k];
}

template <typename T, bool LO16 = false>
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
  Pops<T> q;
  gather<true, T, true, true, LO16>(B, p, x, y, q);
  if (f) {
    double f0 = (double)q.f[0];
    if constexpr (std::is_same<T, float>::value) f0 = f0 + (double)q.lo;
    f[k] = f0 + p.phi_ref;
    for (int i = 1; i < 9; ++i) f[i * n + k] = (double)q.f[i];
  }
  if (g)
    for (int i = 0; i < 9; ++i) g[i * n + k] = (double)q.g[i];
  if (Sp) Sp[k] = (double)Spl[(long long)y * p.pitch + x];
}

__global__ __launch_bounds__(256) void k_copy(float4* __restrict__ dst, const float4* __restrict__ src,
                                               long long n) {
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x)
    dst[k] = src[k];
}

}  // namespace lbm
