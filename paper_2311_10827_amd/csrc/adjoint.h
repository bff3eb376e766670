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
//   KA2 (per tile, LDS): lambda_mu += G^T lambda_{grad mu} (transposed
//       isotropic gradient) on the tile and a one-cell ring, then per cell
//       lambda_phi += G^T lambda_{grad phi} + psi''(phi) lambda_mu
//       - kappa L^T lambda_mu and lambda_f_i = (1 - 1/tau_f) lambda_{f*_i}
//       + lambda_phi (phi = sum_i f_i); kappa and beta partials.
// Transposed stencils enumerate, for each direction, the cells whose
// neighbour (periodic wrap or wall mirror) is the target cell, so walls get
// the exact transpose.  Arithmetic and lambda planes are in the state's
// precision (as in the forward step); parameter partials are FP64.
#pragma once
#include "forward.h"

namespace lbm {

constexpr int NTH = 6;  // kappa, beta, alpha, tau_f, nu_A, nu_B

// Cells x with neighbour(x + c) == v along one axis (c in {-1, 0, 1}).
__device__ __forceinline__ int preimages(int v, int c, int n, int wall, int (&out)[2]) {
  if (!wall) {
    const int r = v - c;
    out[0] = r < 0 ? r + n : (r >= n ? r - n : r);
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

// An axis has a single preimage per direction when it is periodic or the
// cell does not touch a wall along it; then the preimage is v - c, wrapped.
__device__ __forceinline__ bool single_pre(int v, int n, int wall) {
  return !wall || (v >= 1 && v <= n - 2);
}
__device__ __forceinline__ int pre1(int v, int c, int n) {
  const int r = v - c;
  return r < 0 ? r + n : (r >= n ? r - n : r);
}

// (G^T w)(v): transposed isotropic gradient of a 2-vector field w = (wx, wy)
// stored as dense planes [ny][nx].
template <typename A = double, typename T>
__device__ __forceinline__ A grad_T(const KP& p, const T* __restrict__ wx, const T* __restrict__ wy, int x,
                                    int y) {
  A acc = A(0);
  if (single_pre(x, p.nx, p.bcx) && single_pre(y, p.ny, p.bcy)) {
    // an axis direction has one non-zero component: read only that plane
#pragma unroll
    for (int d = 1; d < 9; ++d) {
      const unsigned k = (unsigned)(pre1(y, cy_of(d), p.ny) * p.nx + pre1(x, cx_of(d), p.nx));
      const A t = cy_of(d) == 0   ? A(cx_of(d)) * A(wx[k])
                  : cx_of(d) == 0 ? A(cy_of(d)) * A(wy[k])
                                  : A(cx_of(d)) * A(wx[k]) + A(cy_of(d)) * A(wy[k]);
      acc += A(INV_CS2 * w_of(d)) * t;
    }
    return acc;
  }
#pragma unroll
  for (int d = 1; d < 9; ++d) {
    int px[2], py[2];
    const int nxp = preimages(x, cx_of(d), p.nx, p.bcx, px);
    const int nyp = preimages(y, cy_of(d), p.ny, p.bcy, py);
    const A k3 = A(INV_CS2 * w_of(d));
    for (int a = 0; a < nyp; ++a)
      for (int b = 0; b < nxp; ++b) {
        const unsigned k = (unsigned)(py[a] * p.nx + px[b]);
        acc += k3 * (A(cx_of(d)) * A(wx[k]) + A(cy_of(d)) * A(wy[k]));
      }
  }
  return acc;
}

// (L^T w)(v): transposed isotropic Laplacian of a scalar field.
template <typename T>
__device__ __forceinline__ double lap_T(const KP& p, const T* __restrict__ w, int x, int y) {
  double acc = 0.0;
  if (single_pre(x, p.nx, p.bcx) && single_pre(y, p.ny, p.bcy)) {
#pragma unroll
    for (int d = 1; d < 9; ++d)
      acc += (2.0 * INV_CS2 * w_of(d)) *
             (double)w[(unsigned)(pre1(y, cy_of(d), p.ny) * p.nx + pre1(x, cx_of(d), p.nx))];
    return acc - (2.0 * INV_CS2 * (1.0 - w_of(0))) * (double)w[(unsigned)(y * p.nx + x)];
  }
#pragma unroll
  for (int d = 1; d < 9; ++d) {
    int px[2], py[2];
    const int nxp = preimages(x, cx_of(d), p.nx, p.bcx, px);
    const int nyp = preimages(y, cy_of(d), p.ny, p.bcy, py);
    const double l = 2.0 * INV_CS2 * w_of(d);
    for (int a = 0; a < nyp; ++a)
      for (int b = 0; b < nxp; ++b) acc += l * (double)w[(unsigned)(py[a] * p.nx + px[b])];
  }
  return acc - (2.0 * INV_CS2 * (1.0 - w_of(0))) * (double)w[(unsigned)(y * p.nx + x)];
}

// Forward Laplacian of phi from the dphi plane (3x3 with the forward rule).
template <typename A>
__device__ __forceinline__ A lap_fwd(const A (&v)[3][3]) {
  const A c = v[1][1];
  return A(2.0 / 3.0) * (((v[1][2] - c) + (v[1][0] - c)) + ((v[2][1] - c) + (v[0][1] - c))) +
         A(1.0 / 6.0) * (((v[2][2] - c) + (v[2][0] - c)) + ((v[0][2] - c) + (v[0][0] - c)));
}
__device__ __forceinline__ void grad_fwd(const double (&v)[3][3], double& gx, double& gy) {
  gx = (1.0 / 3.0) * (v[1][2] - v[1][0]) + (1.0 / 12.0) * ((v[2][2] - v[2][0]) + (v[0][2] - v[0][0]));
  gy = (1.0 / 3.0) * (v[2][1] - v[0][1]) + (1.0 / 12.0) * ((v[2][2] - v[0][2]) + (v[2][0] - v[0][0]));
}
// psi'(phi) / beta and psi''(phi) / beta for psi = beta (phi - A)^2 (phi - B)^2.
template <typename A>
__device__ __forceinline__ A dpsi_b(const KP& p, A ph) {
  return A(4.0) * (ph - A(p.phiA)) * (ph - A(p.phiB)) * (ph - A(p.phim));
}
template <typename A>
__device__ __forceinline__ A d2psi_b(const KP& p, A ph) {
  const A a = ph - A(p.phiA), b = ph - A(p.phiB), m = ph - A(p.phim);
  return A(4.0) * (a * b + a * m + b * m);
}

// Sum-reduce NV values over the block and add them to out[0..NV) (the
// block owns `out`; launches on one stream never overlap).  The block's sum
// is taken in A: the FP32 adjoint kernels sum their FP32 per-cell terms in
// FP32 (a wave butterfly of one word per step instead of two), and the
// per-tile partials they add to stay FP64 across the steps.
template <int NV, typename A = double>
__device__ __forceinline__ void block_sum_add(double (&v)[NV], double* __restrict__ out) {
  __shared__ A red[16][NV];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  A s[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    A a = (A)v[k];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) a += __shfl_xor(a, d, 64);
    s[k] = a;
  }
  if (lane == 0)
    for (int k = 0; k < NV; ++k) red[wave][k] = s[k];
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = blockDim.x >> 6;
    for (int k = 0; k < NV; ++k) {
      A a = red[0][k];
      for (int w = 1; w < nw; ++w) a += red[w][k];
      out[k] += (double)a;
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
// Arithmetic in the storage type (FP64 for precision 64, FP32 for 32, like
// the forward step it differentiates); parameter partials in FP64.

// What the local vector-Jacobian product leaves at one cell: the final
// adjoint of g and S_prev, and the adjoints of phi, mu, grad phi and grad mu
// that the stencil transposes spread to the neighbours.
template <typename T>
struct KaCell {
  T lg[9], lS;
  T lphi, lmu, lgpx, lgpy, lgmx, lgmy;
};

// Periodic grids (PER): the cell's row y is the same on a whole wave, so
// every access is a scalar base (plane and row, y - 1, y or y + 1 wrapped)
// plus one of three per-lane byte offsets (columns x - 1, x, x + 1 wrapped);
// no wall selects.
struct PerCols {
  unsigned bm, bc, bp;  // 4 * column of x - 1, x, x + 1
  int ym, yp;           // rows y - 1, y + 1
};

template <typename T, bool INIT, bool MRT = false, bool PER = false>
__device__ __forceinline__ void ka_cell(const KP& p, const T* __restrict__ B, const T* __restrict__ dphi,
                                        const T* __restrict__ mupl, const T* __restrict__ lam_in, int x,
                                        int y, KaCell<T>& o, double (&th)[4], const PerCols& pc = PerCols{}) {
  // The adjoint owes no bitwise match to anything: let a * b + c contract.
#pragma clang fp contract(fast)
  using C = T;
  const long long n = (long long)p.nx * p.ny;  // plane stride of the dense planes
  const unsigned kd = (unsigned)(y * p.nx + x);  // n <= INT32_MAX
  const C half = C(0.5), one = C(1.0), three = C(3.0);
  // ---- forward recompute at this cell (FP32 does not read f_0: see below).
  // The snapshot is read once per adjoint step and not again until the next
  // segment's recompute overwrites it: streaming loads, which leave the
  // last-level cache to the adjoint planes that the next step reads back
  // (1024^2 FP32: 0.1109 against 0.1124 ms per adjoint step incl. recompute).
  constexpr bool F0 = !std::is_same<T, float>::value;
  Pops<T> q;
  Nbhd<T> nb;
  // the cell's row, the same on the whole wave (PER)
  const int yr = PER ? __builtin_amdgcn_readfirstlane(y) : y;
  if constexpr (PER) {
    // pull sources x - c_i; the stencils' neighbours x + (dx, dy)
    auto col = [&](int cx) { return cx == 1 ? pc.bm : (cx == -1 ? pc.bp : pc.bc); };
    auto row = [&](int cy) { return cy == 1 ? pc.ym : (cy == -1 ? pc.yp : yr); };
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const long long r = (long long)row(cy_of(i)) * p.pitch;
      if (F0 || i != 0) q.f[i] = ld_nt_at(B + i * p.ps + r, col(cx_of(i)));
      q.g[i] = ld_nt_at(B + (9 + i) * p.ps + r, col(cx_of(i)));
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const long long r = (long long)row(1 - a) * p.pitch;  // a = 0: y - 1
#pragma unroll
      for (int b = 0; b < 3; ++b) {
        nb.ph[a][b] = ld_at(dphi + r, col(1 - b));  // b = 0: x - 1
        nb.mu[a][b] = ld_at(mupl + r, col(1 - b));
      }
    }
  } else {
    gather<true, T, true, F0, false, true>(B, p, x, y, q);
    load_nbhd(p, dphi, mupl, x, y, nb);
  }
  const C phi_ref = C(p.phi_ref);
  C ph3[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) ph3[a][b] = nb.ph[a][b] + phi_ref;
  const auto& mu3 = nb.mu;
  // phi = sum_i f_i, so f^eq_0 - f_0 = sum_{i!=0} f_i - (1 - w_0) alpha mu,
  // which the FP32 forward step uses too: FP32 skips the two planes of f_0.
  // FP64 takes f_0 itself, keeping the tau_f partial, a small sum of large
  // terms, at FP64 rounding of its own operands.
  C f[9];
#pragma unroll
  for (int i = 1; i < 9; ++i) f[i] = q.f[i];
  f[0] = F0 ? C(q.f[0]) + phi_ref : C(0);
  const C s8 = ((f[1] + f[2]) + (f[3] + f[4])) + ((f[5] + f[6]) + (f[7] + f[8]));
  const C* g = q.g;
  const C phi = ph3[1][1], mu = mu3[1][1];
  const C k3 = C(1.0 / 3.0), k12 = C(1.0 / 12.0);
  const C gpx = k3 * (ph3[1][2] - ph3[1][0]) + k12 * ((ph3[2][2] - ph3[2][0]) + (ph3[0][2] - ph3[0][0]));
  const C gpy = k3 * (ph3[2][1] - ph3[0][1]) + k12 * ((ph3[2][2] - ph3[0][2]) + (ph3[2][0] - ph3[0][0]));
  const C gmx = k3 * (mu3[1][2] - mu3[1][0]) + k12 * ((mu3[2][2] - mu3[2][0]) + (mu3[0][2] - mu3[0][0]));
  const C gmy = k3 * (mu3[2][1] - mu3[0][1]) + k12 * ((mu3[2][2] - mu3[0][2]) + (mu3[2][0] - mu3[0][0]));
  const C rs = C(p.rho_slope);
  const C grx = rs * gpx, gry = rs * gpy;
  const C dB = phi - C(p.phiB);
  const C rho = C(p.rhoB) + dB * rs;
  const C nu = visc<C>(p, dB);
  const C tau = half + three * nu;
  const C wg = recip(tau), kG = one - half * wg;
  const C Fx = C(p.gx) - phi * gmx, Fy = C(p.gy) - phi * gmy;
  const C mx = ((g[1] - g[3]) + (g[5] - g[7])) + (g[8] - g[6]);
  const C my = ((g[2] - g[4]) + (g[5] - g[7])) + (g[6] - g[8]);
  const C irho = recip(rho);
  const C ux = (mx + half * Fx) * irho, uy = (my + half * Fy) * irho;
  const C uu = ux * ux + uy * uy;
  const C snz = ((g[1] + g[2]) + (g[3] + g[4])) + ((g[5] + g[6]) + (g[7] + g[8]));
  const C s0 = -C(2.0 / 3.0) * uu;  // s_0(u) = w_0 (-u.u / (2 c_s^2))
  const C C06 = C(CS2 / (1.0 - w_of(0)));
  const C pr = C06 * (snz + half * (ux * grx + uy * gry) + rho * s0);

  // ---- seeds
  C a[9], c[9];
  C lS;
  if (INIT) {
#pragma unroll
    for (int i = 0; i < 9; ++i) a[i] = c[i] = C(0);
  } else if constexpr (PER) {
    // P^T on a periodic grid: lambda_{f*_j}(x) = lambda'_j(x + c_j)
#pragma unroll
    for (int j = 0; j < 9; ++j) {
      const int cx = cx_of(j), cy = cy_of(j);
      const unsigned cb = cx == 1 ? pc.bp : (cx == -1 ? pc.bm : pc.bc);
      const long long r = (long long)(cy == 1 ? pc.yp : (cy == -1 ? pc.ym : yr)) * p.nx;
      a[j] = ld_at(lam_in + j * n + r, cb);
      c[j] = ld_at(lam_in + (9 + j) * n + r, cb);
    }
  } else {
    // P^T: lambda_{f*_j}(x) = lambda'_j(x + c_j) if that link is fluid,
    // else lambda'_opp(j)(x) (the bounce-back image).
#pragma unroll
    for (int j = 0; j < 9; ++j) {
      int tx = x + cx_of(j), ty = y + cy_of(j);
      const bool wall = (p.bcx && (tx < 0 || tx >= p.nx)) || (p.bcy && (ty < 0 || ty >= p.ny));
      tx = tx < 0 ? tx + p.nx : (tx >= p.nx ? tx - p.nx : tx);
      ty = ty < 0 ? ty + p.ny : (ty >= p.ny ? ty - p.ny : ty);
      const unsigned k = wall ? kd : (unsigned)(ty * p.nx + tx);
      const auto la = wall ? uni(lam_in + opp_of(j) * n) : uni(lam_in + j * n);
      const auto lc = wall ? uni(lam_in + (9 + opp_of(j)) * n) : uni(lam_in + (9 + j) * n);
      a[j] = la[k];
      c[j] = lc[k];
    }
  }
  if constexpr (PER)
    lS = ld_at(lam_in + 18 * n + (long long)yr * p.nx, pc.bc);
  else
    lS = uni(lam_in + 18 * n)[kd];  // S_prev(n+1) = S(n): no streaming

  // ---- order-parameter collision: f* = f - w_f (f - f^eq) + w b (3/2 S - 1/2 S_prev)
  // (MRT: f* = f + R_f (f^eq - f) + ..., R = M^-1 S M, which is symmetric for
  // an orthogonal basis, so lambda_{f^eq} = R_f lambda_{f*})
  const C wf = C(p.omega_f), alpha = C(p.alpha);
  C swb = C(0), lwf = C(0), qeq = C(0);
  C af[9];  // lambda_{f^eq}
  C dfe[9];  // f^eq - f (MRT)
  if constexpr (MRT) {
    C rate[9];
    mrt_rates_f(p, wf, rate);
    mrt_relax<C, false>(rate, a, a, af);
  } else {
#pragma unroll
    for (int i = 0; i < 9; ++i) af[i] = wf * a[i];
  }
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    swb += C(w_of(i) * src_bracket(i)) * a[i];
    const C dfi = i != 0 ? C(w_of(i)) * alpha * mu - f[i]
                  : F0   ? (phi - C(1.0 - w_of(0)) * alpha * mu) - f[0]
                         : s8 - C(1.0 - w_of(0)) * alpha * mu;
    if constexpr (MRT)
      dfe[i] = dfi;
    else
      lwf += a[i] * dfi;
    qeq += C(i == 0 ? -(1.0 - w_of(0)) : w_of(i)) * af[i];
  }
  if constexpr (MRT) {
    // w_f is the rate of the phi and j moments: d/dw_f = sum over them of
    // (M a)_k (M (f^eq - f))_k / |row k|^2
    C ma[9], md[9];
    mom_fwd(a, ma);
    mom_fwd(dfe, md);
    lwf = ma[0] * md[0] * C(1.0 / 9) + (ma[3] * md[3] + ma[5] * md[5]) * C(1.0 / 6);
  }
  C lphi = af[0];           // d f^eq_0 / d phi = 1
  const C lmu = alpha * qeq;
  th[0] += (double)(mu * qeq);          // d/d alpha
  th[1] += (double)(-(wf * wf) * lwf);  // d/d tau_f through 1/tau_f
  const C lSt = lS + C(1.5) * swb;
  const C lSp_out = -half * swb;

  // ---- hydrodynamic collision: g* = g - w_g (g - g^eq) + k_G G~
  // (MRT: g* = g + R_g (g^eq - g) + (I - R_g/2) G~, so lambda_{g^eq} = R_g c
  // and lambda_{G~} = c - R_g c / 2)
  C lwg = C(0), lkG = C(0), lp = C(0), lrho = C(0);
  C lux = C(0), luy = C(0), lFx = C(0), lFy = C(0), lgrx = C(0), lgry = C(0);
  C cg[9];           // lambda_{g^eq}
  C dge[9], Gtv[9];  // g^eq - g and G~ (MRT)
  if constexpr (MRT) {
    C rate[9];
    mrt_rates_g(p, wg, rate);
    mrt_relax<C, false>(rate, c, c, cg);
  } else {
#pragma unroll
    for (int i = 0; i < 9; ++i) cg[i] = wg * c[i];
  }
  if constexpr (!MRT) {
    // BGK: lambda_{g^eq} = w_g c and lambda_{G~} = k_G c, so every sum over
    // the links below is a combination of the weighted lattice moments
    // sum_i w_i c_i {1, c_x, c_y, c_x^2, c_x c_y, c_y^2} of the seed c.
    const C ax = (c[1] + c[3]), ay = (c[2] + c[4]), dsum = (c[5] + c[6]) + (c[7] + c[8]);
    const C w1 = C(1.0 / 9), w5 = C(1.0 / 36);
    const C m0 = C(4.0 / 9) * c[0] + w1 * (ax + ay) + w5 * dsum;
    const C mx = w1 * (c[1] - c[3]) + w5 * ((c[5] - c[6]) + (c[8] - c[7]));
    const C my = w1 * (c[2] - c[4]) + w5 * ((c[5] + c[6]) - (c[7] + c[8]));
    const C mxx = w1 * ax + w5 * dsum, myy = w1 * ay + w5 * dsum;
    const C mxy = w5 * ((c[5] + c[7]) - (c[6] + c[8]));
    // sum_i c_i s_i(u) (eq. Siu) and sum_i c_i g_i
    const C cs = three * (ux * mx + uy * my) +
                 C(4.5) * (ux * ux * mxx + C(2) * ux * uy * mxy + uy * uy * myy) - C(1.5) * uu * m0;
    C cgsum = c[0] * g[0];
#pragma unroll
    for (int i = 1; i < 9; ++i) cgsum += c[i] * g[i];
    // d/dw_g: sum_i c_i (g^eq_i - g_i), g^eq_i = p pw_i + rho s_i, pw_i = 3 (w_i - [i = 0])
    lwg = pr * three * (m0 - c[0]) + rho * cs - cgsum;
    // d/dk_G: sum_i c_i G~_i, G~_i = 3 w_i (c_i.F + (c_i.u)(c_i.grad rho))
    lkG = three * (Fx * mx + Fy * my +
                   (ux * grx * mxx + (ux * gry + uy * grx) * mxy + uy * gry * myy));
    // through g^eq (lambda_{g^eq} = w_g c)
    lp = wg * three * (m0 - c[0]);
    lrho = wg * cs;
    const C rw = rho * wg;
    lux = rw * (three * mx + C(9) * (ux * mxx + uy * mxy) - three * ux * m0);
    luy = rw * (three * my + C(9) * (ux * mxy + uy * myy) - three * uy * m0);
    // through G~ (lambda_{G~} = k_G c)
    const C k3 = three * kG;
    lFx = k3 * mx;
    lFy = k3 * my;
    lux += k3 * (grx * mxx + gry * mxy);
    luy += k3 * (grx * mxy + gry * myy);
    lgrx = k3 * (ux * mxx + uy * mxy);
    lgry = k3 * (ux * mxy + uy * myy);
  } else {
  #pragma unroll
    for (int i = 0; i < 9; ++i) {
      const C cxi = C(cx_of(i)), cyi = C(cy_of(i)), wi = C(w_of(i));
      const C cu = cxi * ux + cyi * uy;
      const C cF = cxi * Fx + cyi * Fy;
      const C cr = cxi * grx + cyi * gry;
      const C si = wi * (three * cu + C(4.5) * cu * cu - C(1.5) * uu);
      const C pw = C(INV_CS2 * (w_of(i) - (i == 0 ? 1.0 : 0.0)));
      const C geq = pr * pw + rho * si;
      const C Gt = three * wi * (cF + cu * cr);
      if constexpr (MRT) {
        dge[i] = geq - g[i];
        Gtv[i] = Gt;
      } else {
        lwg += c[i] * (geq - g[i]);
        lkG += c[i] * Gt;
      }
      const C lgeq = cg[i];
      lp += lgeq * pw;
      lrho += lgeq * si;
      const C rl = rho * lgeq * wi;
      lux += rl * (three * cxi + C(9.0) * cu * cxi - three * ux);
      luy += rl * (three * cyi + C(9.0) * cu * cyi - three * uy);
      const C kc = (MRT ? c[i] - half * cg[i] : kG * c[i]) * three * wi;
      lFx += kc * cxi;
      lFy += kc * cyi;
      lux += kc * cr * cxi;
      luy += kc * cr * cyi;
      lgrx += kc * cu * cxi;
      lgry += kc * cu * cyi;
    }
  }
  // tau_g = 1/2 + 3 nu(phi); w_g = 1/tau_g; k_G = 1 - w_g/2 (MRT: w_g is the
  // rate of j, p_xx and p_xy, in S and in I - S/2)
  if constexpr (MRT) {
    C mc[9], md[9], mG[9];
    mom_fwd(c, mc);
    mom_fwd(dge, md);
    mom_fwd(Gtv, mG);
    lwg = (mc[3] * md[3] + mc[5] * md[5]) * C(1.0 / 6) + (mc[7] * md[7] + mc[8] * md[8]) * C(0.25);
    lkG = (mc[3] * mG[3] + mc[5] * mG[5]) * C(1.0 / 6) + (mc[7] * mG[7] + mc[8] * mG[8]) * C(0.25);
  }
  const C lwg_t = lwg - half * lkG;
  const C lnu = three * (-(wg * wg) * lwg_t);
  C dnu_phi, dnu_A, dnu_B;
  visc_partials<C>(p, dB, nu, dnu_phi, dnu_A, dnu_B);
  lphi += lnu * dnu_phi;
  th[2] += (double)(lnu * dnu_A);
  th[3] += (double)(lnu * dnu_B);
  // S = u . grad phi
  lux += lSt * gpx;
  luy += lSt * gpy;
  C lgpx = lSt * ux, lgpy = lSt * uy;
  // p = C06 (snz + u.grad(rho)/2 + rho s_0(u)), s_0 = -(2/3) |u|^2
  const C lsnz = C06 * lp;
  lux += C06 * lp * (half * grx - C(4.0 / 3.0) * rho * ux);
  luy += C06 * lp * (half * gry - C(4.0 / 3.0) * rho * uy);
  lgrx += C06 * lp * half * ux;
  lgry += C06 * lp * half * uy;
  lrho += C06 * lp * s0;
  // rho u = m + F/2
  const C lmx = lux * irho, lmy = luy * irho;
  lFx += half * lmx;
  lFy += half * lmy;
  lrho += -(lux * ux + luy * uy) * irho;
  // F = -phi grad mu + G
  lphi += -(lFx * gmx + lFy * gmy);
  const C lgmx = -phi * lFx, lgmy = -phi * lFy;
  // rho(phi) and grad rho = rho_slope grad phi
  lphi += rs * lrho;
  lgpx += rs * lgrx;
  lgpy += rs * lgry;

  // ---- outputs
#pragma unroll
  for (int i = 0; i < 9; ++i)
    o.lg[i] = (MRT ? c[i] - cg[i] : (one - wg) * c[i]) + C(cx_of(i)) * lmx + C(cy_of(i)) * lmy +
              (i ? lsnz : C(0));
  o.lS = INIT ? C(0) : lSp_out;
  o.lphi = lphi;
  o.lmu = lmu;
  o.lgpx = lgpx;
  o.lgpy = lgpy;
  o.lgmx = lgmx;
  o.lgmy = lgmy;
}

template <typename T, bool INIT, bool MRT = false, bool PER = false>
__global__ __launch_bounds__(256) void ka_local(const KP p, const T* __restrict__ B,
                                                 const T* __restrict__ dphi,
                                                 const T* __restrict__ mupl,
                                                 const T* __restrict__ lam_in, T* __restrict__ lam_out,
                                                 AdjWork<T> w, double* __restrict__ th_part,
                                                 int ntx) {
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int x = (tile % ntx) * K2_TX + (threadIdx.x & (K2_TX - 1));
  // a tile row is one wave (K2_TX = 64): y is uniform over the wave
  const int y = (tile / ntx) * K2_TY + __builtin_amdgcn_readfirstlane(threadIdx.x / K2_TX);
  double th[4] = {0.0, 0.0, 0.0, 0.0};  // alpha, tau_f, nu_A, nu_B
  if (x < p.nx && y < p.ny) {
    const long long n = (long long)p.nx * p.ny;
    const unsigned kd = (unsigned)(y * p.nx + x);
    KaCell<T> o;
    if constexpr (PER) {
      PerCols pc;
      pc.bm = (unsigned)((x > 0 ? x - 1 : p.nx - 1) * sizeof(T));
      pc.bp = (unsigned)((x < p.nx - 1 ? x + 1 : 0) * sizeof(T));
      pc.bc = (unsigned)(x * sizeof(T));
      // (readfirstlane: the compiler then keeps the row arithmetic, and
      // the row bases of all accesses, in scalar registers)
      pc.ym = __builtin_amdgcn_readfirstlane(y > 0 ? y - 1 : p.ny - 1);
      pc.yp = __builtin_amdgcn_readfirstlane(y < p.ny - 1 ? y + 1 : 0);
      ka_cell<T, INIT, MRT, true>(p, B, dphi, mupl, lam_in, x, y, o, th, pc);
      const long long r = (long long)__builtin_amdgcn_readfirstlane(y) * p.nx;
#pragma unroll
      for (int i = 0; i < 9; ++i) st_at<false>(lam_out + (9 + i) * n + r, pc.bc, o.lg[i]);
      st_at<false>(lam_out + 18 * n + r, pc.bc, o.lS);
      st_at<false>(w.lphi + r, pc.bc, o.lphi);
      st_at<false>(w.lmu + r, pc.bc, o.lmu);
      st_at<false>(w.lgpx + r, pc.bc, o.lgpx);
      st_at<false>(w.lgpy + r, pc.bc, o.lgpy);
      st_at<false>(w.lgmx + r, pc.bc, o.lgmx);
      st_at<false>(w.lgmy + r, pc.bc, o.lgmy);
    } else {
      ka_cell<T, INIT, MRT>(p, B, dphi, mupl, lam_in, x, y, o, th);
#pragma unroll
      for (int i = 0; i < 9; ++i) uni(lam_out + (9 + i) * n)[kd] = o.lg[i];
      uni(lam_out + 18 * n)[kd] = o.lS;
      uni(w.lphi)[kd] = o.lphi;
      uni(w.lmu)[kd] = o.lmu;
      uni(w.lgpx)[kd] = o.lgpx;
      uni(w.lgpy)[kd] = o.lgpy;
      uni(w.lgmx)[kd] = o.lgmx;
      uni(w.lgmy)[kd] = o.lgmy;
    }
  }
  block_sum_add<4, T>(th, th_part + (long long)tile * NTH + 2);
}

// ------------------------------------------------------------- KA2 + KA3
// One pass: lambda_mu_tot = lambda_mu + G^T lambda_{grad mu} on the tile plus
// a one-cell ring, staged in LDS, then lambda_phi and lambda_f on the tile.
// L^T reads lambda_mu_tot at the preimages of the target, which lie at
// offsets {-c} (and {0} for a mirrored wall link) from it: inside the ring.
__device__ __forceinline__ int pre_off(int v, int c, int n, int wall, int (&out)[2]) {
  if (!wall) {
    out[0] = -c;
    return 1;
  }
  if (c == 0) {
    out[0] = 0;
    return 1;
  }
  int k = 0;
  if (c == 1) {
    if (v - 1 >= 0) out[k++] = -1;
    if (v == n - 1) out[k++] = 0;
  } else {
    if (v + 1 <= n - 1) out[k++] = 1;
    if (v == 0) out[k++] = 0;
  }
  return k;
}

// Tiles of KM_TX x KM_TY cells (KM_THREADS threads, KM_TY / (KM_THREADS /
// KM_TX) rows each): the one-cell ring of lambda_mu_tot, recomputed by each
// tile, is 16 % of the tile's cells.
constexpr int KM_TX = 64, KM_TY = 16, KM_THREADS = 256;

template <typename T, bool INIT, bool MRT = false>
__global__ __launch_bounds__(KM_THREADS) void ka_mu_phi(const KP p, const T* __restrict__ dphi,
                                                  const T* __restrict__ lam_in, T* __restrict__ lam_out,
                                                  AdjWork<T> w, double* __restrict__ th_part, int ntx) {
  // The adjoint owes no bitwise match to anything: let a * b + c contract.
#pragma clang fp contract(fast)
  using C = T;  // arithmetic in the storage type, as in ka_local
  constexpr int LW = KM_TX + 2, LH = KM_TY + 2;
  __shared__ C mt[LH][LW];
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  const int x0 = (tile % ntx) * KM_TX, y0 = (tile / ntx) * KM_TY;
  if (!p.bcx && !p.bcy) {
    // Periodic grid: every ring entry has one preimage per direction.  All
    // entries' loads are issued before any is used, so the fill costs one
    // memory round trip instead of one per entry.
    constexpr int NE = (LH * LW + KM_THREADS - 1) / KM_THREADS;
    C lm[NE], gxv[NE][8], gyv[NE][8];
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const int k = min((int)threadIdx.x + e * KM_THREADS, LH * LW - 1);
      const int ly = k / LW, lx = k - ly * LW;
      const int gx = stencil_idx(x0 + lx - 1, p.nx, 0), gy = stencil_idx(y0 + ly - 1, p.ny, 0);
      // the preimages gx - c_x, gy - c_y: three columns and three rows
      const unsigned cx3[3] = {(unsigned)pre1(gx, 1, p.nx), (unsigned)gx, (unsigned)pre1(gx, -1, p.nx)};
      const unsigned ry3[3] = {(unsigned)(pre1(gy, 1, p.ny) * p.nx), (unsigned)(gy * p.nx),
                               (unsigned)(pre1(gy, -1, p.ny) * p.nx)};
      lm[e] = w.lmu[ry3[1] + cx3[1]];
#pragma unroll
      for (int d = 1; d < 9; ++d) {
        const unsigned kk = ry3[1 - cy_of(d)] + cx3[1 - cx_of(d)];
        gxv[e][d - 1] = cx_of(d) != 0 ? w.lgmx[kk] : C(0);
        gyv[e][d - 1] = cy_of(d) != 0 ? w.lgmy[kk] : C(0);
      }
    }
#pragma unroll
    for (int e = 0; e < NE; ++e) {
      const int k = (int)threadIdx.x + e * KM_THREADS;
      if (k < LH * LW) {
        // the sum of grad_T, term by term
        C acc = C(0);
#pragma unroll
        for (int d = 1; d < 9; ++d) {
          const C t = cy_of(d) == 0   ? C(cx_of(d)) * gxv[e][d - 1]
                      : cx_of(d) == 0 ? C(cy_of(d)) * gyv[e][d - 1]
                                      : C(cx_of(d)) * gxv[e][d - 1] + C(cy_of(d)) * gyv[e][d - 1];
          acc += C(INV_CS2 * w_of(d)) * t;
        }
        const int ly = k / LW, lx = k - ly * LW;
        mt[ly][lx] = lm[e] + acc;
      }
    }
  } else {
    for (int k = threadIdx.x; k < LH * LW; k += blockDim.x) {
      const int ly = k / LW, lx = k - ly * LW;
      int gx = x0 + lx - 1, gy = y0 + ly - 1;
      C v = C(0);
      const bool outx = gx < 0 || gx >= p.nx, outy = gy < 0 || gy >= p.ny;
      if (!((outx && p.bcx) || (outy && p.bcy))) {
        gx = stencil_idx(gx, p.nx, 0);
        gy = stencil_idx(gy, p.ny, 0);
        v = w.lmu[(unsigned)(gy * p.nx + gx)] + grad_T<C>(p, w.lgmx, w.lgmy, gx, gy);
      }
      mt[ly][lx] = v;
    }
  }
  __syncthreads();
  const long long n = (long long)p.nx * p.ny;
  const int tx = threadIdx.x & (KM_TX - 1);
  const int x = x0 + tx;
  double th[2] = {0.0, 0.0};  // kappa, beta
  const C k1 = C(1.0 - p.omega_f);
  if (!p.bcx && !p.bcy) {
    // Periodic grid: one preimage per direction everywhere.  The loads of
    // a thread's next row are issued before the current row's arithmetic
    // and stores, so consecutive rows overlap their memory latency.
    struct RowIn {
      C v[3][3];           // phi - phi_ref around the cell
      C lphi;
      C gpx[8], gpy[8];    // lambda_{grad phi} at the preimages (G^T)
      C a[9];              // lambda_{f*}: the transposed pull of lam_in
    };
    // A thread keeps its column (x, clamped on ragged tiles: columns and
    // rows beyond the grid load a valid cell and are not stored) and takes
    // rows that are the same on its whole wave: every access is a scalar
    // base (plane and row) plus one of three per-lane byte offsets.
    const int xc = min(x, p.nx - 1);
    const unsigned cb[3] = {(unsigned)(pre1(xc, 1, p.nx) * sizeof(C)), (unsigned)(xc * sizeof(C)),
                            (unsigned)(pre1(xc, -1, p.nx) * sizeof(C))};  // x - 1, x, x + 1
    auto load_row = [&](int ty, RowIn& in) {
      const int y = __builtin_amdgcn_readfirstlane(min(y0 + ty, p.ny - 1));
      const int ys[3] = {__builtin_amdgcn_readfirstlane(pre1(y, 1, p.ny)), y,
                         __builtin_amdgcn_readfirstlane(pre1(y, -1, p.ny))};  // y - 1, y, y + 1
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) in.v[a][b] = ld_at(dphi + (long long)ys[a] * p.pitch, cb[b]);
      in.lphi = ld_at(w.lphi + (long long)y * p.nx, cb[1]);
#pragma unroll
      for (int d = 1; d < 9; ++d) {  // preimage x - c_d
        const long long r = (long long)ys[1 - cy_of(d)] * p.nx;
        in.gpx[d - 1] = cx_of(d) != 0 ? ld_at(w.lgpx + r, cb[1 - cx_of(d)]) : C(0);
        in.gpy[d - 1] = cy_of(d) != 0 ? ld_at(w.lgpy + r, cb[1 - cx_of(d)]) : C(0);
      }
#pragma unroll
      for (int j = 0; j < 9; ++j) {  // transposed pull: x + c_j
        in.a[j] = C(0);
        if (!INIT) in.a[j] = ld_at(lam_in + j * n + (long long)ys[1 + cy_of(j)] * p.nx, cb[1 + cx_of(j)]);
      }
    };
    auto finish_row = [&](int ty, RowIn& in) {
      const int y = y0 + ty;
      if (x >= p.nx || y >= p.ny) return;
      const long long ry = (long long)y * p.nx;
      const int lx = tx + 1, ly = ty + 1;
      const C lmt = mt[ly][lx];
      C lt = C(0);
#pragma unroll
      for (int d = 1; d < 9; ++d) lt += C(2.0 * INV_CS2 * w_of(d)) * mt[ly - cy_of(d)][lx - cx_of(d)];
      lt -= C(2.0 * INV_CS2 * (1.0 - w_of(0))) * lmt;
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) in.v[a][b] += C(p.phi_ref);
      const C ph = in.v[1][1];
      th[0] += (double)(-lap_fwd<C>(in.v) * lmt);  // mu = psi'(phi) - kappa lap(phi)
      th[1] += (double)(dpsi_b<C>(p, ph) * lmt);
      C gt = C(0);  // G^T lambda_{grad phi}, term by term as in grad_T
#pragma unroll
      for (int d = 1; d < 9; ++d) {
        const C t = cy_of(d) == 0   ? C(cx_of(d)) * in.gpx[d - 1]
                    : cx_of(d) == 0 ? C(cy_of(d)) * in.gpy[d - 1]
                                    : C(cx_of(d)) * in.gpx[d - 1] + C(cy_of(d)) * in.gpy[d - 1];
        gt += C(INV_CS2 * w_of(d)) * t;
      }
      const C lphi = in.lphi + gt + C(p.beta4 * 0.25) * d2psi_b<C>(p, ph) * lmt - C(p.kappa) * lt;
      if constexpr (MRT) {
        C rate[9], ra[9];  // lambda_f = (I - R_f) lambda_{f*} + lambda_phi
        mrt_rates_f(p, C(p.omega_f), rate);
        mrt_relax<C, false>(rate, in.a, in.a, ra);
#pragma unroll
        for (int j = 0; j < 9; ++j) st_at<false>(lam_out + j * n + ry, cb[1], (in.a[j] - ra[j]) + lphi);
      } else {
#pragma unroll
        for (int j = 0; j < 9; ++j) st_at<false>(lam_out + j * n + ry, cb[1], k1 * in.a[j] + lphi);
      }
    };
    constexpr int NR = KM_TY / (KM_THREADS / KM_TX);  // rows per thread
    // a tile row is one wave (KM_TX = 64)
    const int ty0 = __builtin_amdgcn_readfirstlane(threadIdx.x / KM_TX);
    RowIn in[2];
    load_row(ty0, in[0]);
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if (r + 1 < NR) load_row(ty0 + (r + 1) * (KM_THREADS / KM_TX), in[(r + 1) & 1]);
      finish_row(ty0 + r * (KM_THREADS / KM_TX), in[r & 1]);
    }
  } else {
    for (int ty = threadIdx.x / KM_TX; ty < KM_TY; ty += KM_THREADS / KM_TX) {
      const int y = y0 + ty;
      if (x >= p.nx || y >= p.ny) continue;
      const unsigned kd = (unsigned)(y * p.nx + x);
      const int lx = tx + 1, ly = ty + 1;
      const C lmt = mt[ly][lx];
      // L^T lambda_mu_tot from LDS
      C lt = C(0);
      if (single_pre(x, p.nx, p.bcx) && single_pre(y, p.ny, p.bcy)) {
#pragma unroll
        for (int d = 1; d < 9; ++d) lt += C(2.0 * INV_CS2 * w_of(d)) * mt[ly - cy_of(d)][lx - cx_of(d)];
      } else {
#pragma unroll
        for (int d = 1; d < 9; ++d) {
          int ox[2], oy[2];
          const int nxo = pre_off(x, cx_of(d), p.nx, p.bcx, ox);
          const int nyo = pre_off(y, cy_of(d), p.ny, p.bcy, oy);
          for (int a = 0; a < nyo; ++a)
            for (int b = 0; b < nxo; ++b) lt += C(2.0 * INV_CS2 * w_of(d)) * mt[ly + oy[a]][lx + ox[b]];
        }
      }
      lt -= C(2.0 * INV_CS2 * (1.0 - w_of(0))) * lmt;
      // forward phi around the cell for lap(phi) and psi
      C v[3][3];
      const int xs[3] = {stencil_idx(x - 1, p.nx, p.bcx), x, stencil_idx(x + 1, p.nx, p.bcx)};
      const int ys[3] = {stencil_idx(y - 1, p.ny, p.bcy), y, stencil_idx(y + 1, p.ny, p.bcy)};
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) v[a][b] = dphi[(unsigned)(ys[a] * p.pitch + xs[b])] + C(p.phi_ref);
      const C ph = v[1][1];
      th[0] += (double)(-lap_fwd<C>(v) * lmt);  // mu = psi'(phi) - kappa lap(phi)
      th[1] += (double)(dpsi_b<C>(p, ph) * lmt);
      const C lphi = w.lphi[kd] + grad_T<C>(p, w.lgpx, w.lgpy, x, y) +
                     C(p.beta4 * 0.25) * d2psi_b<C>(p, ph) * lmt - C(p.kappa) * lt;
      C av[9];
#pragma unroll
      for (int j = 0; j < 9; ++j) {
        C a = C(0);
        if (!INIT) {
          int qx = x + cx_of(j), qy = y + cy_of(j);
          const bool wall = (p.bcx && (qx < 0 || qx >= p.nx)) || (p.bcy && (qy < 0 || qy >= p.ny));
          qx = qx < 0 ? qx + p.nx : (qx >= p.nx ? qx - p.nx : qx);
          qy = qy < 0 ? qy + p.ny : (qy >= p.ny ? qy - p.ny : qy);
          const unsigned k = wall ? kd : (unsigned)(qy * p.nx + qx);
          const auto la = wall ? uni(lam_in + opp_of(j) * n) : uni(lam_in + j * n);
          a = la[k];
        }
        av[j] = a;
      }
      if constexpr (MRT) {
        C rate[9], ra[9];  // lambda_f = (I - R_f) lambda_{f*} + lambda_phi
        mrt_rates_f(p, C(p.omega_f), rate);
        mrt_relax<C, false>(rate, av, av, ra);
#pragma unroll
        for (int j = 0; j < 9; ++j) uni(lam_out + j * n)[kd] = (av[j] - ra[j]) + lphi;
      } else {
#pragma unroll
        for (int j = 0; j < 9; ++j) uni(lam_out + j * n)[kd] = k1 * av[j] + lphi;
      }
    }
  }
  block_sum_add<2, T>(th, th_part + (long long)tile * NTH + 0);
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
    dphi0[kd] = (double)w.lphi[kd] + p.beta4 * 0.25 * d2psi_b<double>(p, v[1][1]) * lm -
                p.kappa * lap_T(p, w.lmu_tot, x, y);
    th[0] = -lap_fwd<double>(v) * lm;
    th[1] = dpsi_b<double>(p, v[1][1]) * lm;
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
