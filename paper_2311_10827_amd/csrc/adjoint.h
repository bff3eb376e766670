// Hand-written adjoint (reverse mode) of one time step of the well-balanced
// phase-field LBM, and of the initialisation.
//
// The state at time n is s_n = (f, g, S_prev): pre-collision populations and
// the previous-step convection source.  One step is
//   s_{n+1} = P(collide(s_n)),     S_prev(n+1) = S(s_n),
// with P the pull streaming (periodic wrap or half-way bounce-back).  Given
// lambda_{n+1} (the gradient of a loss with respect to s_{n+1}) the kernels
// below compute lambda_n = (d s_{n+1} / d s_n)^T lambda_{n+1} and add
// (d s_{n+1} / d theta)^T lambda_{n+1} to per-tile parameter partials, for
// theta = (kappa, beta, alpha, tau_f, nu_A, nu_B).
//
//   KA1 (per cell): transposed streaming P^T of lambda (a gather with the
//       opposite offsets: no atomics), then the local vector-Jacobian product
//       of the collision and of u, p, S, F, rho, nu.  The g adjoint is local
//       and written directly; lambda for phi, mu, grad phi and grad mu goes to
//       work planes.
//   KA2 (per cell): lambda_mu += G^T lambda_{grad mu} (transposed isotropic
//       gradient), plus the kappa and beta partials.
//   KA3 (per cell): lambda_phi += G^T lambda_{grad phi} + psi''(phi) lambda_mu
//       - kappa L^T lambda_mu, then lambda_f_i = (1 - 1/tau_f) lambda_{f*_i}
//       + lambda_phi (phi = sum_i f_i).
// Transposed stencils enumerate, for each direction, the cells whose
// neighbour (periodic wrap or wall mirror) is the target cell, so walls get
// the exact transpose.  Arithmetic is FP64; lambda planes are stored in the
// state's precision.
#pragma once
#include "forward.h"

namespace lbm {

constexpr int NTH = 6;  // kappa, beta, alpha, tau_f, nu_A, nu_B

// Cells x with neighbour(x + c) == v along one axis (c in {-1, 0, 1}).
__device__ __forceinline__ int preimages(int v, int c, int n, int wall, int (&out)[2]) {
  if (!wall) {
    int r = (v - c) % n;
    out[0] = r < 0 ? r + n : r;
    return 1;
  }
  if (c == 0) {
    out[0] = v;
    return 1;
  }
  int k = 0;
  if (c == 1) {
    if (v - 1 >= 0) out[k++] = v - 1;
    if (v == n - 1) out[k++] = n - 1;
  } else {
    if (v + 1 <= n - 1) out[k++] = v + 1;
    if (v == 0) out[k++] = 0;
  }
  return k;
}

// (G^T w)(v): transposed isotropic gradient of a 2-vector field w = (wx, wy)
// stored as dense planes [ny][nx].
template <typename T>
__device__ __forceinline__ double grad_T(const KP& p, const T* __restrict__ wx, const T* __restrict__ wy,
                                         int x, int y) {
  double acc = 0.0;
#pragma unroll
  for (int d = 1; d < 9; ++d) {
    int px[2], py[2];
    const int nxp = preimages(x, cx_of(d), p.nx, p.bcx, px);
    const int nyp = preimages(y, cy_of(d), p.ny, p.bcy, py);
    const double k3 = INV_CS2 * w_of(d);
    for (int a = 0; a < nyp; ++a)
      for (int b = 0; b < nxp; ++b) {
        const long long k = (long long)py[a] * p.nx + px[b];
        acc += k3 * ((double)cx_of(d) * (double)wx[k] + (double)cy_of(d) * (double)wy[k]);
      }
  }
  return acc;
}

// (L^T w)(v): transposed isotropic Laplacian of a scalar field.
template <typename T>
__device__ __forceinline__ double lap_T(const KP& p, const T* __restrict__ w, int x, int y) {
  double acc = 0.0;
#pragma unroll
  for (int d = 1; d < 9; ++d) {
    int px[2], py[2];
    const int nxp = preimages(x, cx_of(d), p.nx, p.bcx, px);
    const int nyp = preimages(y, cy_of(d), p.ny, p.bcy, py);
    const double l = 2.0 * INV_CS2 * w_of(d);
    for (int a = 0; a < nyp; ++a)
      for (int b = 0; b < nxp; ++b) acc += l * (double)w[(long long)py[a] * p.nx + px[b]];
  }
  return acc - (2.0 * INV_CS2 * (1.0 - w_of(0))) * (double)w[(long long)y * p.nx + x];
}

// Forward Laplacian of phi from the dphi plane (3x3 with the forward rule).
__device__ __forceinline__ double lap_fwd(const double (&v)[3][3]) {
  const double c = v[1][1];
  return (2.0 / 3.0) * (((v[1][2] - c) + (v[1][0] - c)) + ((v[2][1] - c) + (v[0][1] - c))) +
         (1.0 / 6.0) * (((v[2][2] - c) + (v[2][0] - c)) + ((v[0][2] - c) + (v[0][0] - c)));
}
__device__ __forceinline__ void grad_fwd(const double (&v)[3][3], double& gx, double& gy) {
  gx = (1.0 / 3.0) * (v[1][2] - v[1][0]) + (1.0 / 12.0) * ((v[2][2] - v[2][0]) + (v[0][2] - v[0][0]));
  gy = (1.0 / 3.0) * (v[2][1] - v[0][1]) + (1.0 / 12.0) * ((v[2][2] - v[0][2]) + (v[2][0] - v[0][0]));
}
// psi'(phi) / beta and psi''(phi) / beta for psi = beta (phi - A)^2 (phi - B)^2.
__device__ __forceinline__ double dpsi_b(const KP& p, double ph) {
  return 4.0 * (ph - p.phiA) * (ph - p.phiB) * (ph - p.phim);
}
__device__ __forceinline__ double d2psi_b(const KP& p, double ph) {
  const double a = ph - p.phiA, b = ph - p.phiB, m = ph - p.phim;
  return 4.0 * (a * b + a * m + b * m);
}

// Sum-reduce NV values over the block and add them to out[0..NV) (the
// block owns `out`; launches on one stream never overlap).
template <int NV>
__device__ __forceinline__ void block_sum_add(double (&v)[NV], double* __restrict__ out) {
  __shared__ double red[16][NV];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double a = v[k];
#pragma unroll
    for (int s = 32; s >= 1; s >>= 1) a += __shfl_xor(a, s, 64);
    v[k] = a;
  }
  if (lane == 0)
    for (int k = 0; k < NV; ++k) red[wave][k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = blockDim.x >> 6;
    for (int k = 0; k < NV; ++k) {
      double a = red[0][k];
      for (int w = 1; w < nw; ++w) a += red[w][k];
      out[k] += a;
    }
  }
}

// Adjoint work planes (dense [ny][nx], storage type T).
template <typename T>
struct AdjWork {
  T *lphi, *lmu, *lgpx, *lgpy, *lgmx, *lgmy, *lmu_tot;
};

// ------------------------------------------------------------------ KA1
// INIT: the map is s_0 -> S_prev(0) = S(s_0) only (no collision, no
// streaming); the seed is lambda of S_prev(0) and lambda_f*, lambda_g* = 0.
template <typename T, bool INIT>
__global__ __launch_bounds__(256) void ka_local(const KP p, const T* __restrict__ B,
                                                 const T* __restrict__ Spl,
                                                 const T* __restrict__ dphi,
                                                 const T* __restrict__ mupl,
                                                 const T* __restrict__ lam_in, T* __restrict__ lam_out,
                                                 AdjWork<T> w, double* __restrict__ th_part,
                                                 int ntx) {
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int x = (tile % ntx) * K2_TX + (threadIdx.x & (K2_TX - 1));
  const int y = (tile / ntx) * K2_TY + threadIdx.x / K2_TX;
  double th[4] = {0.0, 0.0, 0.0, 0.0};  // alpha, tau_f, nu_A, nu_B
  if (x < p.nx && y < p.ny) {
    const long long n = (long long)p.nx * p.ny;
    const long long kd = (long long)y * p.nx + x;
    const long long o = (long long)y * p.pitch + x;
    // ---- forward recompute at this cell (FP64)
    Pops<T> q;
    gather<true>(B, p, x, y, q);
    Nbhd<T> nb;
    load_nbhd(p, dphi, mupl, x, y, nb);
    double ph3[3][3], mu3[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        ph3[a][b] = (double)nb.ph[a][b] + p.phi_ref;
        mu3[a][b] = (double)nb.mu[a][b];
      }
    double f[9], g[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      f[i] = (double)q.f[i];
      g[i] = (double)q.g[i];
    }
    if constexpr (std::is_same<T, float>::value) f[0] += (double)q.lo;
    f[0] += p.phi_ref;
    const double phi = ph3[1][1], mu = mu3[1][1];
    double gpx, gpy, gmx, gmy;
    grad_fwd(ph3, gpx, gpy);
    grad_fwd(mu3, gmx, gmy);
    const double rs = p.rho_slope;
    const double grx = rs * gpx, gry = rs * gpy;
    const double dB = phi - p.phiB;
    const double rho = p.rhoB + dB * rs;
    const double nu = p.nuB + dB * p.nu_slope;
    const double tau = 0.5 + INV_CS2 * nu;
    const double wg = 1.0 / tau, kG = 1.0 - 0.5 * wg;
    const double Fx = p.gx - phi * gmx, Fy = p.gy - phi * gmy;
    const double mx = ((g[1] - g[3]) + (g[5] - g[7])) + (g[8] - g[6]);
    const double my = ((g[2] - g[4]) + (g[5] - g[7])) + (g[6] - g[8]);
    const double ux = (mx + 0.5 * Fx) / rho, uy = (my + 0.5 * Fy) / rho;
    const double uu = ux * ux + uy * uy;
    const double snz = ((g[1] + g[2]) + (g[3] + g[4])) + ((g[5] + g[6]) + (g[7] + g[8]));
    const double s0 = -(2.0 / 3.0) * uu;  // s_0(u) = w_0 (-u.u / (2 c_s^2))
    const double C06 = CS2 / (1.0 - w_of(0));
    const double pr = C06 * (snz + 0.5 * (ux * grx + uy * gry) + rho * s0);

    // ---- seeds
    double a[9], c[9];
    double lS;
    if (INIT) {
#pragma unroll
      for (int i = 0; i < 9; ++i) a[i] = c[i] = 0.0;
      lS = (double)lam_in[18 * n + kd];
    } else {
      // P^T: lambda_{f*_j}(x) = lambda'_j(x + c_j) if that link is fluid,
      // else lambda'_opp(j)(x) (the bounce-back image).
#pragma unroll
      for (int j = 0; j < 9; ++j) {
        int tx = x + cx_of(j), ty = y + cy_of(j);
        bool wall = (p.bcx && (tx < 0 || tx >= p.nx)) || (p.bcy && (ty < 0 || ty >= p.ny));
        long long k;
        int pl;
        if (wall) {
          k = kd;
          pl = opp_of(j);
        } else {
          tx = tx < 0 ? tx + p.nx : (tx >= p.nx ? tx - p.nx : tx);
          ty = ty < 0 ? ty + p.ny : (ty >= p.ny ? ty - p.ny : ty);
          k = (long long)ty * p.nx + tx;
          pl = j;
        }
        a[j] = (double)lam_in[pl * n + k];
        c[j] = (double)lam_in[(9 + pl) * n + k];
      }
      lS = (double)lam_in[18 * n + kd];  // S_prev(n+1) = S(n), no streaming
    }

    // ---- order-parameter collision: f* = f - w_f (f - f^eq) + w b (3/2 S - 1/2 S_prev)
    const double wf = p.omega_f;
    double swb = 0.0, lwf = 0.0, qeq = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      swb += w_of(i) * src_bracket(i) * a[i];
      const double feq = i == 0 ? phi - (1.0 - w_of(0)) * p.alpha * mu : w_of(i) * p.alpha * mu;
      lwf += a[i] * (feq - f[i]);
      qeq += (i == 0 ? -(1.0 - w_of(0)) : w_of(i)) * (wf * a[i]);
    }
    double lphi = wf * a[0];       // d f^eq_0 / d phi = 1
    const double lmu = p.alpha * qeq;
    th[0] += mu * qeq;             // d/d alpha
    th[1] += -(wf * wf) * lwf;     // d/d tau_f through 1/tau_f
    const double lSt = lS + 1.5 * swb;
    const double lSp_out = -0.5 * swb;

    // ---- hydrodynamic collision: g* = g - w_g (g - g^eq) + k_G G~
    double lwg = 0.0, lkG = 0.0, lp = 0.0, lrho = 0.0;
    double lux = 0.0, luy = 0.0, lFx = 0.0, lFy = 0.0, lgrx = 0.0, lgry = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const double cxi = cx_of(i), cyi = cy_of(i), wi = w_of(i);
      const double cu = cxi * ux + cyi * uy;
      const double cF = cxi * Fx + cyi * Fy;
      const double cr = cxi * grx + cyi * gry;
      const double si = wi * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
      const double geq = (pr * INV_CS2) * (wi - (i == 0 ? 1.0 : 0.0)) + rho * si;
      lwg += c[i] * (geq - g[i]);
      const double Gt = 3.0 * wi * (cF + cu * cr);
      lkG += c[i] * Gt;
      const double lgeq = wg * c[i];
      lp += lgeq * INV_CS2 * (wi - (i == 0 ? 1.0 : 0.0));
      lrho += lgeq * si;
      const double rl = rho * lgeq * wi;
      lux += rl * (3.0 * cxi + 9.0 * cu * cxi - 3.0 * ux);
      luy += rl * (3.0 * cyi + 9.0 * cu * cyi - 3.0 * uy);
      const double kc = kG * c[i] * 3.0 * wi;
      lFx += kc * cxi;
      lFy += kc * cyi;
      lux += kc * cr * cxi;
      luy += kc * cr * cyi;
      lgrx += kc * cu * cxi;
      lgry += kc * cu * cyi;
    }
    // tau_g = 1/2 + 3 nu(phi); w_g = 1/tau_g; k_G = 1 - w_g/2
    const double lwg_t = lwg - 0.5 * lkG;
    const double lnu = INV_CS2 * (-(wg * wg) * lwg_t);
    lphi += lnu * p.nu_slope;
    const double t = dB / (p.phiA - p.phiB);
    th[2] += lnu * t;
    th[3] += lnu * (1.0 - t);
    // S = u . grad phi
    lux += lSt * gpx;
    luy += lSt * gpy;
    double lgpx = lSt * ux, lgpy = lSt * uy;
    // p = C06 (snz + u.grad(rho)/2 + rho s_0(u)), s_0 = -(2/3) |u|^2
    const double lsnz = C06 * lp;
    lux += C06 * lp * (0.5 * grx - (4.0 / 3.0) * rho * ux);
    luy += C06 * lp * (0.5 * gry - (4.0 / 3.0) * rho * uy);
    lgrx += C06 * lp * 0.5 * ux;
    lgry += C06 * lp * 0.5 * uy;
    lrho += C06 * lp * s0;
    // rho u = m + F/2
    const double lmx = lux / rho, lmy = luy / rho;
    lFx += 0.5 * lmx;
    lFy += 0.5 * lmy;
    lrho += -(lux * ux + luy * uy) / rho;
    // F = -phi grad mu + G
    lphi += -(lFx * gmx + lFy * gmy);
    const double lgmx = -phi * lFx, lgmy = -phi * lFy;
    // rho(phi) and grad rho = rho_slope grad phi
    lphi += rs * lrho;
    lgpx += rs * lgrx;
    lgpy += rs * lgry;

    // ---- outputs
#pragma unroll
    for (int i = 0; i < 9; ++i)
      lam_out[(9 + i) * n + kd] = (T)((1.0 - wg) * c[i] + (double)cx_of(i) * lmx +
                                      (double)cy_of(i) * lmy + (i ? lsnz : 0.0));
    lam_out[18 * n + kd] = (T)(INIT ? 0.0 : lSp_out);
    w.lphi[kd] = (T)lphi;
    w.lmu[kd] = (T)lmu;
    w.lgpx[kd] = (T)lgpx;
    w.lgpy[kd] = (T)lgpy;
    w.lgmx[kd] = (T)lgmx;
    w.lgmy[kd] = (T)lgmy;
    (void)o;
  }
  block_sum_add<4>(th, th_part + (long long)tile * NTH + 2);
}

// ------------------------------------------------------------------ KA2
template <typename T>
__global__ __launch_bounds__(256) void ka_mu(const KP p, const T* __restrict__ dphi, AdjWork<T> w,
                                              double* __restrict__ th_part, int ntx) {
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int x = (tile % ntx) * K2_TX + (threadIdx.x & (K2_TX - 1));
  const int y = (tile / ntx) * K2_TY + threadIdx.x / K2_TX;
  double th[2] = {0.0, 0.0};  // kappa, beta
  if (x < p.nx && y < p.ny) {
    const long long kd = (long long)y * p.nx + x;
    const double lmt = (double)w.lmu[kd] + grad_T(p, w.lgmx, w.lgmy, x, y);
    w.lmu_tot[kd] = (T)lmt;
    double v[3][3];
    const int xs[3] = {stencil_idx(x - 1, p.nx, p.bcx), x, stencil_idx(x + 1, p.nx, p.bcx)};
    const int ys[3] = {stencil_idx(y - 1, p.ny, p.bcy), y, stencil_idx(y + 1, p.ny, p.bcy)};
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) v[a][b] = (double)dphi[(long long)ys[a] * p.pitch + xs[b]] + p.phi_ref;
    th[0] = -lap_fwd(v) * lmt;           // mu = psi'(phi) - kappa lap(phi)
    th[1] = dpsi_b(p, v[1][1]) * lmt;
  }
  block_sum_add<2>(th, th_part + (long long)tile * NTH + 0);
}

// ------------------------------------------------------------------ KA3
// lambda_f_i = (1 - w_f) lambda_{f*_i} + lambda_phi.  INIT: lambda_{f*} = 0.
template <typename T, bool INIT>
__global__ __launch_bounds__(256) void ka_phi(const KP p, const T* __restrict__ dphi,
                                               const T* __restrict__ lam_in, T* __restrict__ lam_out,
                                               AdjWork<T> w, int ntx) {
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int x = (tile % ntx) * K2_TX + (threadIdx.x & (K2_TX - 1));
  const int y = (tile / ntx) * K2_TY + threadIdx.x / K2_TX;
  if (x >= p.nx || y >= p.ny) return;
  const long long n = (long long)p.nx * p.ny;
  const long long kd = (long long)y * p.nx + x;
  const double ph = (double)dphi[(long long)y * p.pitch + x] + p.phi_ref;
  const double lmt = (double)w.lmu_tot[kd];
  const double lphi = (double)w.lphi[kd] + grad_T(p, w.lgpx, w.lgpy, x, y) +
                      p.beta4 * 0.25 * d2psi_b(p, ph) * lmt - p.kappa * lap_T(p, w.lmu_tot, x, y);
  const double k1 = 1.0 - p.omega_f;
#pragma unroll
  for (int j = 0; j < 9; ++j) {
    double a = 0.0;
    if (!INIT) {
      int tx = x + cx_of(j), ty = y + cy_of(j);
      bool wall = (p.bcx && (tx < 0 || tx >= p.nx)) || (p.bcy && (ty < 0 || ty >= p.ny));
      if (wall) {
        a = (double)lam_in[opp_of(j) * n + kd];
      } else {
        tx = tx < 0 ? tx + p.nx : (tx >= p.nx ? tx - p.nx : tx);
        ty = ty < 0 ? ty + p.ny : (ty >= p.ny ? ty - p.ny : ty);
        a = (double)lam_in[j * n + (long long)ty * p.nx + tx];
      }
    }
    lam_out[j * n + kd] = (T)(k1 * a + lphi);
  }
}

// ---------------------------------------------------- initialisation adjoint
// f(0) = f^eq(phi0, mu0) with mu0 = mu(phi0), g(0) = g^eq(0, 0) = 0 (no phi0
// dependence).  lam_f: total adjoint of f(0) (seed plus the S_prev(0) path).
// KI1: lambda_phi0 (local part) and lambda_mu0; KI2: the mu0 stencil.
template <typename T>
__global__ __launch_bounds__(256) void ki_local(const KP p, const double* __restrict__ phi0,
                                                 const T* __restrict__ mupl,
                                                 const T* __restrict__ lam0,
                                                 const T* __restrict__ lf_s, AdjWork<T> w,
                                                 double* __restrict__ th_part, int ntx) {
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int x = (tile % ntx) * K2_TX + (threadIdx.x & (K2_TX - 1));
  const int y = (tile / ntx) * K2_TY + threadIdx.x / K2_TX;
  double th[1] = {0.0};
  if (x < p.nx && y < p.ny) {
    const long long n = (long long)p.nx * p.ny;
    const long long kd = (long long)y * p.nx + x;
    const double mu0 = (double)mupl[(long long)y * p.pitch + x];
    double lf[9];
    for (int i = 0; i < 9; ++i) lf[i] = (double)lam0[i * n + kd] + (double)lf_s[i * n + kd];
    double q = -(1.0 - w_of(0)) * lf[0];
    for (int i = 1; i < 9; ++i) q += w_of(i) * lf[i];
    w.lphi[kd] = (T)lf[0];
    w.lmu_tot[kd] = (T)(p.alpha * q);
    th[0] = mu0 * q;
    (void)phi0;
  }
  block_sum_add<1>(th, th_part + (long long)tile * NTH + 2);
}

template <typename T>
__global__ __launch_bounds__(256) void ki_phi(const KP p, const double* __restrict__ phi0, AdjWork<T> w,
                                               double* __restrict__ dphi0, double* __restrict__ th_part,
                                               int ntx) {
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int x = (tile % ntx) * K2_TX + (threadIdx.x & (K2_TX - 1));
  const int y = (tile / ntx) * K2_TY + threadIdx.x / K2_TX;
  double th[2] = {0.0, 0.0};
  if (x < p.nx && y < p.ny) {
    const long long kd = (long long)y * p.nx + x;
    double v[3][3];
    const int xs[3] = {stencil_idx(x - 1, p.nx, p.bcx), x, stencil_idx(x + 1, p.nx, p.bcx)};
    const int ys[3] = {stencil_idx(y - 1, p.ny, p.bcy), y, stencil_idx(y + 1, p.ny, p.bcy)};
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) v[a][b] = phi0[(long long)ys[a] * p.nx + xs[b]];
    const double lm = (double)w.lmu_tot[kd];
    dphi0[kd] = (double)w.lphi[kd] + p.beta4 * 0.25 * d2psi_b(p, v[1][1]) * lm -
                p.kappa * lap_T(p, w.lmu_tot, x, y);
    th[0] = -lap_fwd(v) * lm;
    th[1] = dpsi_b(p, v[1][1]) * lm;
  }
  block_sum_add<2>(th, th_part + (long long)tile * NTH + 0);
}

__global__ __launch_bounds__(256) void k_sum_theta(const double* __restrict__ part, long long n,
                                                    double* __restrict__ out) {
  // one block; fixed assignment of tiles to lanes
  double v[NTH] = {0, 0, 0, 0, 0, 0};
  for (long long b = threadIdx.x; b < n; b += blockDim.x)
    for (int k = 0; k < NTH; ++k) v[k] += part[b * NTH + k];
  for (int k = 0; k < NTH; ++k) out[k] = 0.0;
  __syncthreads();
  block_sum_add<NTH>(v, out);
}

__global__ __launch_bounds__(256) void k_zero(double* __restrict__ a, long long n) {
  for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n;
       k += (long long)gridDim.x * blockDim.x)
    a[k] = 0.0;
}

}  // namespace lbm
