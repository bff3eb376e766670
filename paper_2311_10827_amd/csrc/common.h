// Device-side building blocks shared by the kernels of liblbmwb: D2Q9
// tables, kernel parameters, tile order, neighbour indexing, the pull gather
// and the fixed-order diagnostic reduction.
//
// Population storage (one "pop buffer"), planes of the storage type T:
//   FP64: 18 planes  f_0..f_8, g_0..g_8
//   FP32: 19 planes  f_0(hi), f_1..f_8, g_0..g_8, f_0(lo)
// In FP32 the rest population of the order-parameter distribution is kept as
// an unevaluated sum hi + lo (minus phi_ref): it is of order one and changes
// by far less than an FP32 ulp per step, so a single FP32 word would drop
// those changes.  hi is an FP32 word; lo, never more than half an ulp of hi,
// is an FP32 word or, for states larger than 1 GiB (the kernels' LO16
// template argument), a 16-bit multiple of ulp(hi)/2^16 in the first half of
// its plane (see lo_encode).  All other populations are small
// deviations from the rest equilibrium (g^eq(p=0, u=0) = 0, f^eq_i(mu=0) = 0
// for i != 0) and keep full relative precision in one FP32 word.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <type_traits>

namespace lbm {

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
constexpr double CS2 = 1.0 / 3.0;   // c_s^2
constexpr double INV_CS2 = 3.0;     // 1 / c_s^2, exact
// Source shape of Sec. 2.3.1, eq. F_i: -1 + I:(c_i c_i - c_s^2 I)/(2 c_s^2),
// with I:(c c - c_s^2 I) = |c|^2 - 2 c_s^2 in two dimensions.
__host__ __device__ constexpr double src_bracket(int i) {
  return -1.0 + 0.5 * ((double)(cx_of(i) * cx_of(i) + cy_of(i) * cy_of(i)) - 2.0 * CS2) * INV_CS2;
}

template <typename T>
struct Store;
template <>
struct Store<double> {
  static constexpr int NB = 18;  // planes per pop buffer
};
template <>
struct Store<float> {
  static constexpr int NB = 19;  // plus the low word of f_0
};
constexpr int LO_PLANE = 18;
constexpr int NQ = 11;  // diagnostic quantities, in the order of lbm_diag's leading fields

// Kernel parameters: geometry and the constants of the step in FP64; the
// FP32 kernels convert them once.
struct KP {
  int nx, ny, pitch, bcx, bcy;
  long long ps;                 // plane stride, elements
  double phi_ref;               // stored offset of phi and f_0 (0 in FP64)
  double phiA, phiB, phim;
  double beta4;                 // 4 beta
  double kappa, alpha;
  double omega_f;               // 1 / tau_f
  double rhoB, rho_slope;       // rho = rho_B + (phi - phi_B) rho_slope
  double nuB, nu_slope;         // nu  = nu_B  + (phi - phi_B) nu_slope (linear form)
  double gx, gy;
  int nu_form;                  // NU_LINEAR, NU_INVERSE or NU_EXP
  double dphiAB;                // phi_A - phi_B
  double nuA, ln_nuA, ln_nuB;   // for the inverse-linear and exponential forms
  double nu_dphi;               // d nu/d phi over nu^2 (inverse) or over nu (exponential)
  double inv_nuA, inv_nuB;      // 1/nu_A, 1/nu_B
  int collision;                // 0 BGK, 1 MRT
  double mf[4];                 // MRT rates of f: e, eps, q, p
  double mg[2];                 // MRT rates of g: (rho, e, eps), q
};

// ---------------------------------------------------------------- MRT basis
// Orthogonal D2Q9 moment basis of Lallemand and Luo,
// m = (rho, e, eps, j_x, q_x, j_y, q_y, p_xx, p_xy) = M v, from the
// polynomials 1, 3|c|^2 - 4, (9|c|^4 - 21|c|^2 + 8)/2, c_x, (3|c|^2 - 5) c_x,
// c_y, (3|c|^2 - 5) c_y, c_x^2 - c_y^2, c_x c_y of the lattice velocities.
template <typename C>
__device__ __forceinline__ void mom_fwd(const C (&v)[9], C (&m)[9]) {
  const C a = (v[1] + v[2]) + (v[3] + v[4]);  // axis links
  const C d = (v[5] + v[6]) + (v[7] + v[8]);  // diagonal links
  m[0] = v[0] + a + d;
  m[1] = C(-4) * v[0] - a + C(2) * d;
  m[2] = C(4) * v[0] - C(2) * a + d;
  const C jxa = v[1] - v[3], jxd = (v[5] - v[6]) + (v[8] - v[7]);
  const C jya = v[2] - v[4], jyd = (v[5] + v[6]) - (v[7] + v[8]);
  m[3] = jxa + jxd;
  m[4] = C(-2) * jxa + jxd;
  m[5] = jya + jyd;
  m[6] = C(-2) * jya + jyd;
  m[7] = (v[1] + v[3]) - (v[2] + v[4]);
  m[8] = (v[5] + v[7]) - (v[6] + v[8]);
}
// v = M^-1 m = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12, 1/4, 1/4) m
// (the rows of M are orthogonal with those squared norms).
template <typename C>
__device__ __forceinline__ void mom_inv(const C (&m)[9], C (&v)[9]) {
  const C r = m[0] * C(1.0 / 9), e = m[1] * C(1.0 / 36), ep = m[2] * C(1.0 / 36);
  const C jx = m[3] * C(1.0 / 6), qx = m[4] * C(1.0 / 12), jy = m[5] * C(1.0 / 6),
          qy = m[6] * C(1.0 / 12), pxx = m[7] * C(0.25), pxy = m[8] * C(0.25);
  v[0] = r - C(4) * e + C(4) * ep;
  const C ax = r - e - C(2) * ep, dg = r + C(2) * e + ep;
  const C hx = jx - C(2) * qx, hy = jy - C(2) * qy;  // axis: j - 2q
  const C sx = jx + qx, sy = jy + qy;                // diagonal: j + q
  v[1] = ax + hx + pxx;
  v[2] = ax + hy - pxx;
  v[3] = ax - hx + pxx;
  v[4] = ax - hy - pxx;
  v[5] = dg + sx + sy + pxy;
  v[6] = dg - sx + sy - pxy;
  v[7] = dg - sx - sy + pxy;
  v[8] = dg + sx - sy - pxy;
}
// MRT relaxation, moment by moment: out = M^-1 (rate (M d) + (1 - rate/2) (M b));
// with HAS_B false, b is not read and its term is left out.
template <typename C, bool HAS_B>
__device__ __forceinline__ void mrt_relax(const C (&rate)[9], const C (&d)[9], const C (&b)[9],
                                          C (&out)[9]) {
  C md[9], m[9];
  mom_fwd(d, md);
  if constexpr (HAS_B) {
    C mb[9];
    mom_fwd(b, mb);
#pragma unroll
    for (int k = 0; k < 9; ++k) m[k] = rate[k] * md[k] + (C(1) - C(0.5) * rate[k]) * mb[k];
  } else {
#pragma unroll
    for (int k = 0; k < 9; ++k) m[k] = rate[k] * md[k];
  }
  mom_inv(m, out);
}
// Rates per moment (rho, e, eps, j_x, q_x, j_y, q_y, p_xx, p_xy).  f: the
// fluxes (and the conserved phi) at 1/tau_f; g: the fluxes and stresses at
// 1/tau_g, rho, e and eps at one common rate (p is recovered from
// sum_{i!=0} g_i = (8 rho + e - eps)/9, which unequal rates would disturb).
template <typename C>
__device__ __forceinline__ void mrt_rates_f(const KP& p, C wf, C (&r)[9]) {
  r[0] = wf; r[1] = C(p.mf[0]); r[2] = C(p.mf[1]); r[3] = wf; r[4] = C(p.mf[2]);
  r[5] = wf; r[6] = C(p.mf[2]); r[7] = C(p.mf[3]); r[8] = C(p.mf[3]);
}
template <typename C>
__device__ __forceinline__ void mrt_rates_g(const KP& p, C wg, C (&r)[9]) {
  r[0] = C(p.mg[0]); r[1] = C(p.mg[0]); r[2] = C(p.mg[0]); r[3] = wg; r[4] = C(p.mg[1]);
  r[5] = wg; r[6] = C(p.mg[1]); r[7] = wg; r[8] = wg;
}

// The forward step takes MRT as the BGK update plus a correction on the
// moments whose rate differs from the BGK rate w:
//   M^-1 S M d = w d + M^-1 (S - w) M d,
// and with the forcing, M^-1 [S M d + (I - S/2) M G]
//   = w d + (1 - w/2) G + M^-1 (S - w) M (d - G/2).
// f: S - w is nonzero on e, eps, q_x, q_y, p_xx, p_xy.
template <typename C>
__device__ __forceinline__ void mrt_corr_f(const KP& p, C w, const C (&d)[9], C (&out)[9]) {
  const C a = (d[1] + d[2]) + (d[3] + d[4]), dd = (d[5] + d[6]) + (d[7] + d[8]);
  const C jxa = d[1] - d[3], jxd = (d[5] - d[6]) + (d[8] - d[7]);
  const C jya = d[2] - d[4], jyd = (d[5] + d[6]) - (d[7] + d[8]);
  const C e = (C(-4) * d[0] - a + C(2) * dd) * ((C(p.mf[0]) - w) * C(1.0 / 36));
  const C ep = (C(4) * d[0] - C(2) * a + dd) * ((C(p.mf[1]) - w) * C(1.0 / 36));
  const C kq = (C(p.mf[2]) - w) * C(1.0 / 12), kp = (C(p.mf[3]) - w) * C(0.25);
  const C qx = (C(-2) * jxa + jxd) * kq, qy = (C(-2) * jya + jyd) * kq;
  const C pxx = ((d[1] + d[3]) - (d[2] + d[4])) * kp, pxy = ((d[5] + d[7]) - (d[6] + d[8])) * kp;
  out[0] = C(4) * (ep - e);
  const C ax = -e - C(2) * ep, dg = C(2) * e + ep;
  out[1] = ax - C(2) * qx + pxx;
  out[2] = ax - C(2) * qy - pxx;
  out[3] = ax + C(2) * qx + pxx;
  out[4] = ax + C(2) * qy - pxx;
  out[5] = dg + qx + qy + pxy;
  out[6] = dg - qx + qy - pxy;
  out[7] = dg - qx - qy + pxy;
  out[8] = dg + qx - qy - pxy;
}
// g: S - w is nonzero on rho, e, eps (rate mg[0]) and q_x, q_y (mg[1]); z is
// d - G/2.
template <typename C>
__device__ __forceinline__ void mrt_corr_g(const KP& p, C w, const C (&z)[9], C (&out)[9]) {
  const C a = (z[1] + z[2]) + (z[3] + z[4]), dd = (z[5] + z[6]) + (z[7] + z[8]);
  const C jxa = z[1] - z[3], jxd = (z[5] - z[6]) + (z[8] - z[7]);
  const C jya = z[2] - z[4], jyd = (z[5] + z[6]) - (z[7] + z[8]);
  const C kpr = C(p.mg[0]) - w, kq = (C(p.mg[1]) - w) * C(1.0 / 12);
  const C r = (z[0] + a + dd) * (kpr * C(1.0 / 9));
  const C e = (C(-4) * z[0] - a + C(2) * dd) * (kpr * C(1.0 / 36));
  const C ep = (C(4) * z[0] - C(2) * a + dd) * (kpr * C(1.0 / 36));
  const C qx = (C(-2) * jxa + jxd) * kq, qy = (C(-2) * jya + jyd) * kq;
  out[0] = r - C(4) * e + C(4) * ep;
  const C ax = r - e - C(2) * ep, dg = r + C(2) * e + ep;
  out[1] = ax - C(2) * qx;
  out[2] = ax - C(2) * qy;
  out[3] = ax + C(2) * qx;
  out[4] = ax + C(2) * qy;
  out[5] = dg + qx + qy;
  out[6] = dg - qx + qy;
  out[7] = dg - qx - qy;
  out[8] = dg + qx - qy;
}

// Viscosity across the interface (Sec. 2.3.2).  The paper adopts nu linear in
// phi (eq. vis); it names the inverse-linear and the exponential forms as the
// alternatives, read here as 1/nu, respectively ln nu, linear in the phase-A
// fraction s = (phi - phi_B)/(phi_A - phi_B).
enum { NU_LINEAR = 0, NU_INVERSE = 1, NU_EXP = 2 };

// nu at a cell from dB = phi - phi_B.  The form is uniform over a launch.
template <typename C>
__device__ __forceinline__ C visc(const KP& p, C dB) {
  if (p.nu_form == NU_LINEAR) return C(p.nuB) + dB * C(p.nu_slope);
  const C s = dB / C(p.dphiAB);
  if (p.nu_form == NU_INVERSE) return C(1) / (s / C(p.nuA) + (C(1) - s) / C(p.nuB));
  const C e = s * C(p.ln_nuA) + (C(1) - s) * C(p.ln_nuB);
  if constexpr (std::is_same<C, float>::value)
    return expf(e);
  else
    return exp(e);
}

// d nu/d phi, d nu/d nu_A and d nu/d nu_B at a cell, from dB and nu = visc(dB).
template <typename C>
__device__ __forceinline__ void visc_partials(const KP& p, C dB, C nu, C& d_phi, C& d_A, C& d_B) {
  const C s = dB * C(1.0 / p.dphiAB);
  if (p.nu_form == NU_LINEAR) {
    d_phi = C(p.nu_slope);
    d_A = s;
    d_B = C(1) - s;
  } else if (p.nu_form == NU_INVERSE) {  // nu = 1/q, q = s/nu_A + (1 - s)/nu_B
    const C n2 = nu * nu;
    d_phi = n2 * C(p.nu_dphi);
    d_A = n2 * s * C(p.inv_nuA * p.inv_nuA);
    d_B = n2 * (C(1) - s) * C(p.inv_nuB * p.inv_nuB);
  } else {  // ln nu = s ln nu_A + (1 - s) ln nu_B
    d_phi = nu * C(p.nu_dphi);
    d_A = nu * s * C(p.inv_nuA);
    d_B = nu * (C(1) - s) * C(p.inv_nuB);
  }
}

// XCD-aware tile order: the hardware deals workgroups round-robin over the
// 8 XCDs, so each XCD gets one contiguous band of tiles and neighbouring
// tiles share that XCD's L2.  A bijection of [0, n).
__device__ __forceinline__ int xcd_tile(int b, int n) {
  const int X = 8;
  const int per = n / X, rem = n % X;
  const int xcd = b % X, local = b / X;
  return xcd < rem ? xcd * (per + 1) + local : rem * (per + 1) + (xcd - rem) * per + local;
}

// A wave-uniform pointer (a plane base) as a global-memory pointer, passed
// through readfirstlane so that it stays in scalar registers: the compiler
// may then not fold a lane's offset into it, and each access is the base
// plus one vector offset.
template <typename P>
using gmem = __attribute__((address_space(1))) P*;
template <typename P>
__device__ __forceinline__ gmem<P> uni(P* ptr) {
  const unsigned long long v = reinterpret_cast<unsigned long long>(ptr);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  return (gmem<P>)(((unsigned long long)hi << 32) | lo);
}

// Global load and store at a wave-uniform base plus a per-lane byte offset
// (one vector register; the base stays in scalar registers).
template <typename P>
__device__ __forceinline__ P ld_at(const P* base, unsigned byte_off) {
  using G = __attribute__((address_space(1))) const char*;
  const G b = (G)uni(base);
  return *(__attribute__((address_space(1))) const P*)(b + byte_off);
}
template <typename P>
__device__ __forceinline__ P ld_nt_at(const P* base, unsigned byte_off) {
  using G = __attribute__((address_space(1))) const char*;
  const G b = (G)uni(base);
  return __builtin_nontemporal_load((__attribute__((address_space(1))) const P*)(b + byte_off));
}
template <bool NT, typename P>
__device__ __forceinline__ void st_at(P* base, unsigned byte_off, P v) {
  using G = __attribute__((address_space(1))) char*;
  const G b = (G)uni(base);
  __attribute__((address_space(1))) P* ptr = (__attribute__((address_space(1))) P*)(b + byte_off);
  if constexpr (NT)
    __builtin_nontemporal_store(v, ptr);
  else
    *ptr = v;
}

// Stencil neighbour: periodic wrap, or the mirrored adjacent cell across a
// wall.  Valid for any integer v; one period out of range costs a compare,
// the general remainder runs only for lanes farther out.
__device__ __forceinline__ int stencil_idx(int v, int n, int wall) {
  if (wall) return v < 0 ? 0 : (v >= n ? n - 1 : v);
  if (v >= -n && v < 2 * n) return v < 0 ? v + n : (v >= n ? v - n : v);
  int r = v % n;
  return r < 0 ? r + n : r;
}

// Pull sources along one axis for the links arriving at v: m = source of a
// +1 link (v-1), p = source of a -1 link (v+1); -1 marks a wall crossing.
struct PullCols {
  int m, p;
};
__device__ __forceinline__ PullCols pull_cols(int v, int n, int wall) {
  PullCols r;
  r.m = v > 0 ? v - 1 : (wall ? -1 : n - 1);
  r.p = v < n - 1 ? v + 1 : (wall ? -1 : 0);
  return r;
}

// Pre-collision populations of cell (x, y): pull streaming from the buffer,
// half-way bounce-back (B_opp(i) at the cell itself) for links from a wall.
template <typename T>
struct Pops {
  T f[9], g[9];
  T lo;  // FP32 only: low word of f_0
};

// The low word of the FP32 rest population: lo = q ulp(hi) / 2^16 with q a
// 16-bit integer (|lo| <= ulp(hi)/2 keeps |q| <= 2^15), which holds hi + lo
// to about 2^-40 relative in 16 bits where an FP32 word takes 32.  For
// |hi| < 2^-87 no low word is kept.
__device__ __forceinline__ float lo_unit(float hi) {  // ulp(hi) / 2^16 = 2^(e - 166)
  const unsigned e = (__float_as_uint(hi) >> 23) & 0xFFu;  // biased exponent of hi
  return e > 39u ? __uint_as_float((e - 39u) << 23) : 0.0f;
}
__device__ __forceinline__ short lo_encode(float hi, float lo) {
  const unsigned e = (__float_as_uint(hi) >> 23) & 0xFFu;
  if (e <= 39u) return 0;
  const float q = rintf(lo * __uint_as_float((293u - e) << 23));  // lo / unit, exact scaling
  return (short)fminf(fmaxf(q, -32768.0f), 32767.0f);
}
__device__ __forceinline__ float lo_decode(float hi, short q) { return (float)q * lo_unit(hi); }
template <typename T>
__device__ __forceinline__ const short* lo_plane(const T* B, const KP& p) {
  return reinterpret_cast<const short*>(B + LO_PLANE * p.ps);
}
template <typename T>
__device__ __forceinline__ short* lo_plane(T* B, const KP& p) {
  return reinterpret_cast<short*>(B + LO_PLANE * p.ps);
}

// 1/x: in FP32 the hardware reciprocal (1 ulp), in FP64 the division.
template <typename C>
__device__ __forceinline__ C recip(C x) {
  if constexpr (std::is_same<C, float>::value)
    return __builtin_amdgcn_rcpf(x);
  else
    return C(1) / x;
}

// A load, streaming (non-temporal) when NTL.
template <bool NTL, typename T>
__device__ __forceinline__ T load_as(const T* ptr) {
  if constexpr (NTL)
    return __builtin_nontemporal_load(ptr);
  else
    return *ptr;
}

// WITH_G: also gather g.  WITH_F: gather f (and the low word of f_0);
// WITH_F0 = false leaves out f_0 and its low word.  LO16: the FP32 low word
// is stored in 16 bits.  NTL: streaming loads of the populations.
// Offsets within a plane fit in 32 bits (pitch * ny <= INT32_MAX); the
// plane of each load is one of two wave-uniform bases (the direction's own
// or, for a bounce-back lane, the opposite one).
template <bool WITH_G, typename T, bool WITH_F = true, bool WITH_F0 = true, bool LO16 = false, bool NTL = false>
__device__ __forceinline__ void gather(const T* __restrict__ B, const KP& p, int x, int y, Pops<T>& q) {
  const PullCols px = pull_cols(x, p.nx, p.bcx);
  const PullCols py = pull_cols(y, p.ny, p.bcy);
  const unsigned own = (unsigned)(y * p.pitch + x);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int cx = cx_of(i), cy = cy_of(i);
    const int sx = cx == 1 ? px.m : (cx == -1 ? px.p : x);
    const int sy = cy == 1 ? py.m : (cy == -1 ? py.p : y);
    const bool bb = sx < 0 || sy < 0;
    const unsigned off = bb ? own : (unsigned)(sy * p.pitch + sx);
    if (WITH_F && (WITH_F0 || i != 0)) {
      const T* pf = bb ? B + opp_of(i) * p.ps : B + i * p.ps;
      q.f[i] = load_as<NTL>(pf + off);
    }
    if (WITH_G) {
      const T* pg = bb ? B + (9 + opp_of(i)) * p.ps : B + (9 + i) * p.ps;
      q.g[i] = load_as<NTL>(pg + off);
    }
  }
  if constexpr (WITH_F && WITH_F0 && std::is_same<T, float>::value) {
    if constexpr (LO16)
      q.lo = lo_decode(q.f[0], lo_plane(B, p)[own]);
    else
      q.lo = (B + LO_PLANE * p.ps)[own];
  }
}

// Store one pre-collision population so that the pull gather returns it:
// B_i(x - c_i), or B_opp(i)(x) if the link crosses a wall.  Each buffer entry
// is the image of exactly one (cell, direction).
template <typename T>
__device__ __forceinline__ void scatter(T* __restrict__ B, const KP& p, int x, int y, int plane0, int i,
                                        T v) {
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

// Split a value into an FP32 pair hi + lo.
__device__ __forceinline__ void split2(double v, float& hi, float& lo) {
  hi = (float)v;
  lo = (float)(v - (double)hi);
}

// ------------------------------------------------------------ diagnostics
struct Diag {
  double v[NQ];
};
__device__ __forceinline__ void diag_identity(Diag& d) {
  d.v[0] = d.v[1] = d.v[2] = d.v[3] = 0.0;
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

// Fixed-order block reduction: xor butterfly inside each 64-lane
// wavefront, then the block's waves in index order.  Bitwise reproducible.
__device__ inline void block_reduce_write(Diag& d, double* __restrict__ out) {
  __shared__ double red[16][NQ];
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

}  // namespace lbm
