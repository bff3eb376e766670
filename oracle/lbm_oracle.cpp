// Plain, slow FP64 CPU oracle of the well-balanced phase-field lattice
// Boltzmann step (Ju, Liu, Yan, Bao, Sun, Guo; arXiv 2311.10827).
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link,
// load or call this file; only the test-suite, the smoke check and the CPU
// baseline leg of the benchmark use it.  It shares no code, header, table or
// constant with the HIP library: every lattice table and every formula below
// is restated here from the paper.
//
// The method is an iteration, so the oracle takes the algorithm's steps in
// the paper's order and notation, one full-grid pass per step, with no
// fusion or blocking:
//   1. order parameter phi = sum_i f_i                      (Sec. 2.3.1, eq. order-parameter)
//   2. density and viscosity, linear in phi                 (Sec. 2.3.2, eq. vis and the sentence before it;
//      the viscosity optionally in the inverse-linear or exponential form named there)
//   3. chemical potential mu = psi'(phi) - kappa lap(phi)   (Sec. 2.1, eq. chemical_potencial; Sec. 2.3.2, eq. Laplace)
//   4. isotropic gradients of phi, mu and rho               (Sec. 2.3.2, eq. gradient)
//   5. force F = -phi grad(mu) + G                          (Sec. 2.1 after eq. 6; Sec. 2.3.2 after eq. GGi)
//   6. velocity rho u = sum_i c_i g_i + F/2                 (Sec. 2.3.2, macroscopic subequations)
//   7. pressure p                                           (same)
//   8. convection source S = u . grad(phi)                  (Sec. 2.3.1, eq. F_i)
//   9. CH collision with source and its time derivative     (Sec. 2.3.1, eqs. BGK, H_i, F_i)
//  10. NS collision with forcing                            (Sec. 2.3.2, eqs. BGK-NS, G_i, Siu, GGi)
//  11. streaming (periodic, or half-way bounce-back walls)
//  12. keep S for the next step's time derivative of F_i
//
// Readings where the paper is silent or garbled:
//  * c_s^2 = 1/3, delta_x = delta_t = 1 (the text's "c/sqrt(3)" is garbled).
//  * The time derivative in eq. BGK is the first-order backward difference
//    [F_i(t) - F_i(t-1)]/delta_t, which needs S of the previous step.
//  * rho(phi) and nu(phi) are linear between (phi_B, rho_B|nu_B) and
//    (phi_A, rho_A|nu_A); tau_g = 1/2 + nu/c_s^2 per cell (Sec. 2.3.2).
//    The inverse-linear and exponential viscosity forms, which the paper
//    names without writing them out, are read as 1/nu, respectively ln nu,
//    linear in the same phase-A fraction s = (phi - phi_B)/(phi_A - phi_B),
//    with no clamping of s (as for the linear form).
//  * tau_f = 1/2 + M/(c_s^2 alpha) (Sec. 2.3.1, eq. mobility).
//  * Walls: half-way bounce-back for f and g; ghost values of phi and mu
//    across a wall mirror the adjacent cell (the paper's tests are periodic).
//  * Initial state: f = f^eq(phi0, mu(phi0)), g = g^eq(p=0, u0), and the
//    previous-step source equals S computed from that state.
//  * Multiple relaxation times (the paper only says BGK extends to them):
//    both collisions relax the non-equilibrium part in the orthogonal moment
//    basis of Lallemand and Luo, m = (rho, e, eps, j_x, q_x, j_y, q_y, p_xx,
//    p_xy).  f: the fluxes j relax at 1/tau_f (the mobility of eq. mobility),
//    rho at 1/tau_f, the others at given rates; its source is added as in BGK.
//    g: j, p_xx, p_xy relax at 1/tau_g(phi), q at a given rate, and rho, e
//    and eps at one common given rate: in this pressure form p is recovered
//    from sum_{i!=0} g_i = (8 rho + e - eps)/9, which the collision must not
//    change through unequal rates on its parts (with unequal rates even a
//    uniform fluid at rest is unstable).  The forcing of eq. GGi enters in
//    moment space with (I - S/2) in place of the scalar (1 - 1/(2 tau_g)).
//    With every rate equal this is BGK.
//
// The scalar type is a template parameter.  With R = double this is the
// oracle; with R = Dual (value + one tangent) the same code, unchanged, is
// the forward-mode tangent-linear model used to check the hand-written
// adjoint: each arithmetic operation carries its exact derivative.

#include <cmath>
#include <cstdint>
#include <cstring>
#include <cstdlib>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ---------------------------------------------------------------- dual numbers
struct Dual {
  double v, d;
  Dual() : v(0), d(0) {}
  Dual(double a) : v(a), d(0) {}
  Dual(double a, double b) : v(a), d(b) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
  double q = a.v / b.v;
  return Dual(q, (a.d - q * b.d) / b.v);
}
inline Dual operator+(Dual a, double b) { return Dual(a.v + b, a.d); }
inline Dual operator+(double a, Dual b) { return Dual(a + b.v, b.d); }
inline Dual operator-(Dual a, double b) { return Dual(a.v - b, a.d); }
inline Dual operator-(double a, Dual b) { return Dual(a - b.v, -b.d); }
inline Dual operator*(Dual a, double b) { return Dual(a.v * b, a.d * b); }
inline Dual operator*(double a, Dual b) { return Dual(a * b.v, a * b.d); }
inline Dual operator/(Dual a, double b) { return Dual(a.v / b, a.d / b); }
inline Dual operator/(double a, Dual b) {
  double q = a / b.v;
  return Dual(q, -q * b.d / b.v);
}
inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
inline Dual& operator-=(Dual& a, Dual b) { a = a - b; return a; }
inline double val(double a) { return a; }
inline double val(Dual a) { return a.v; }
// exp and ln with their exact derivatives, for the exponential viscosity form
inline double expo(double a) { return std::exp(a); }
inline Dual expo(Dual a) {
  const double e = std::exp(a.v);
  return Dual(e, e * a.d);
}
inline double logn(double a) { return std::log(a); }
inline Dual logn(Dual a) { return Dual(std::log(a.v), a.d / a.v); }

// ------------------------------------------------------------- D2Q9 lattice
// Sec. 2.2, eq. eq:ci and the weights stated just after it.  Order used on
// every interface of this project: 0 rest; 1 (+1,0); 2 (0,+1); 3 (-1,0);
// 4 (0,-1); 5 (+1,+1); 6 (-1,+1); 7 (-1,-1); 8 (+1,-1).
const int Q = 9;
const int CX[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
const int CY[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
const double WT[Q] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                      1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
const double CS2 = 1.0 / 3.0;  // c_s^2 with c = 1
const double INV_CS2 = 3.0;    // 1/c_s^2, exact because c_s^2 = 1/3
int opposite(int i) {
  for (int j = 0; j < Q; ++j)
    if (CX[j] == -CX[i] && CY[j] == -CY[i]) return j;
  return -1;
}

// Orthogonal D2Q9 moment basis (Lallemand and Luo, Phys. Rev. E 61, 6546),
// evaluated from its defining polynomials of the lattice velocity c:
//   1, e = 3|c|^2 - 4, eps = (9|c|^4 - 21|c|^2 + 8)/2, j_x = c_x,
//   q_x = (3|c|^2 - 5) c_x, j_y = c_y, q_y = (3|c|^2 - 5) c_y,
//   p_xx = c_x^2 - c_y^2, p_xy = c_x c_y.
// The rows are orthogonal, so the inverse is the transpose divided by the
// squared row norms.
struct MomentBasis {
  double M[Q][Q];  // [moment][direction]
  double norm2[Q];
  MomentBasis() {
    for (int i = 0; i < Q; ++i) {
      const double cx = CX[i], cy = CY[i], c2 = cx * cx + cy * cy;
      const double row[Q] = {1.0, 3.0 * c2 - 4.0, (9.0 * c2 * c2 - 21.0 * c2 + 8.0) / 2.0,
                             cx, (3.0 * c2 - 5.0) * cx, cy, (3.0 * c2 - 5.0) * cy,
                             cx * cx - cy * cy, cx * cy};
      for (int k = 0; k < Q; ++k) M[k][i] = row[k];
    }
    for (int k = 0; k < Q; ++k) {
      norm2[k] = 0.0;
      for (int i = 0; i < Q; ++i) norm2[k] += M[k][i] * M[k][i];
    }
  }
};
const MomentBasis MB;

}  // namespace

extern "C" {

// Boundary kinds.
enum { ORC_PERIODIC = 0, ORC_WALL = 1 };
// Viscosity across the interface: nu, 1/nu or ln nu linear in phi.
enum { ORC_NU_LINEAR = 0, ORC_NU_INVERSE = 1, ORC_NU_EXP = 2 };
// Collision operator.
enum { ORC_BGK = 0, ORC_MRT = 1 };

typedef struct {
  int32_t nx, ny;
  int32_t bc_x, bc_y;
  double phi_A, phi_B;  // paper phi_l, phi_v
  double rho_A, rho_B;
  double nu_A, nu_B;
  double kappa, beta;
  double M, alpha;      // tau_f = 1/2 + M/(c_s^2 alpha)
  double gx, gy;        // body force G
  int32_t nu_form;      // ORC_NU_*
  int32_t collision;    // ORC_BGK or ORC_MRT
  double mrt_f[4];      // MRT rates of f for e, eps, q, p (p_xx and p_xy)
  double mrt_g[2];      // MRT rates of g for (rho, e, eps) together, and q
} orc_params;

}  // extern "C"

namespace {

template <class R>
struct Theta {       // the differentiable parameters
  R kappa, beta, alpha, tau_f, nu_A, nu_B;
};

template <class R>
struct Sim {
  orc_params p;
  Theta<R> th;
  int nx, ny;
  std::vector<R> f, g, Sp;     // pre-collision populations [9][ny][nx], S of previous step
  // per-step work fields
  std::vector<R> phi, rho, nu, mu, gphx, gphy, gmux, gmuy, grhx, grhy, Fx, Fy, ux, uy, pr, S;
  std::vector<R> fs, gs;       // post-collision populations

  explicit Sim(const orc_params& q) : p(q), nx(q.nx), ny(q.ny) {
    th.kappa = q.kappa;
    th.beta = q.beta;
    th.alpha = q.alpha;
    th.tau_f = 0.5 + q.M * INV_CS2 / q.alpha;  // eq. mobility solved for tau_f
    th.nu_A = q.nu_A;
    th.nu_B = q.nu_B;
    size_t n = (size_t)nx * ny;
    f.assign(Q * n, R(0)); g.assign(Q * n, R(0)); Sp.assign(n, R(0));
    fs.assign(Q * n, R(0)); gs.assign(Q * n, R(0));
    for (auto* v : {&phi, &rho, &nu, &mu, &gphx, &gphy, &gmux, &gmuy, &grhx, &grhy,
                    &Fx, &Fy, &ux, &uy, &pr, &S})
      v->assign(n, R(0));
  }
  size_t cells() const { return (size_t)nx * ny; }
  size_t at(int x, int y) const { return (size_t)y * nx + x; }

  // Index of the neighbour value used by the finite-difference stencils:
  // periodic wrap, or the mirrored adjacent cell across a wall.
  int sx(int x) const {
    if (p.bc_x == ORC_PERIODIC) return ((x % nx) + nx) % nx;
    return x < 0 ? 0 : (x >= nx ? nx - 1 : x);
  }
  int sy(int y) const {
    if (p.bc_y == ORC_PERIODIC) return ((y % ny) + ny) % ny;
    return y < 0 ? 0 : (y >= ny ? ny - 1 : y);
  }

  // Sec. 2.3.2, eq. gradient: grad Psi = sum_{i!=0} w_i c_i Psi(x+c_i) / c_s^2.
  void gradient(const std::vector<R>& psi, std::vector<R>& gx, std::vector<R>& gy) const {
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        R ax = 0.0, ay = 0.0;
        for (int i = 1; i < Q; ++i) {
          R v = psi[at(sx(x + CX[i]), sy(y + CY[i]))];
          ax += WT[i] * CX[i] * v * INV_CS2;
          ay += WT[i] * CY[i] * v * INV_CS2;
        }
        gx[at(x, y)] = ax;
        gy[at(x, y)] = ay;
      }
  }

  // Sec. 2.3.2, eq. Laplace: lap Psi = sum_{i!=0} 2 w_i [Psi(x+c_i) - Psi(x)] / c_s^2.
  void laplacian(const std::vector<R>& psi, std::vector<R>& out) const {
#pragma omp parallel for schedule(static)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        R c = psi[at(x, y)];
        R a = 0.0;
        for (int i = 1; i < Q; ++i)
          a += 2.0 * WT[i] * (psi[at(sx(x + CX[i]), sy(y + CY[i]))] - c) * INV_CS2;
        out[at(x, y)] = a;
      }
  }

  // Sec. 2.1, eq. chemical_potencial, with the discrete Laplacian above.
  void chemical_potential(const std::vector<R>& ph, std::vector<R>& out) const {
    std::vector<R> lap(cells());
    laplacian(ph, lap);
    const double pl = p.phi_A, pv = p.phi_B, pm = 0.5 * (p.phi_A + p.phi_B);
#pragma omp parallel for schedule(static)
    for (long k = 0; k < (long)cells(); ++k)
      out[k] = 4.0 * th.beta * (ph[k] - pl) * (ph[k] - pv) * (ph[k] - pm) - th.kappa * lap[k];
  }

  // Linear density in phi (Sec. 2.3.2, the text before eq. vis):
  // rho = rho_B + (phi - phi_B) (rho_A - rho_B) / (phi_A - phi_B).
  R density(R ph) const {
    const double slope = (p.rho_A - p.rho_B) / (p.phi_A - p.phi_B);
    return p.rho_B + (ph - p.phi_B) * slope;
  }
  // Kinematic viscosity.  Linear in phi as the paper adopts it (eq. vis), the
  // same line as for rho; or one of the two alternatives it names in Sec. 2.3.2
  // (inverse-linear, exponential), written with the phase-A fraction s.
  R viscosity(R ph) const {
    if (p.nu_form == ORC_NU_LINEAR) {
      const R slope = (th.nu_A - th.nu_B) / (p.phi_A - p.phi_B);
      return th.nu_B + (ph - p.phi_B) * slope;
    }
    const R s = (ph - p.phi_B) / (p.phi_A - p.phi_B);
    if (p.nu_form == ORC_NU_INVERSE) return 1.0 / (s / th.nu_A + (1.0 - s) / th.nu_B);
    if (p.nu_form == ORC_NU_EXP) return expo(s * logn(th.nu_A) + (1.0 - s) * logn(th.nu_B));
    std::abort();
  }

  // Sec. 2.3.1, eq. H_i.
  void feq(R ph, R m, R* out) const {
    for (int i = 0; i < Q; ++i)
      out[i] = (i == 0) ? ph - (1.0 - WT[0]) * th.alpha * m : WT[i] * th.alpha * m;
  }
  // Sec. 2.3.1, eq. F_i, for a given value of u . grad(phi).
  void source(R s, R* out) const {
    for (int i = 0; i < Q; ++i) {
      // I : (c_i c_i - c_s^2 I) = |c_i|^2 - 2 c_s^2 in two dimensions
      double contraction = (double)(CX[i] * CX[i] + CY[i] * CY[i]) - 2.0 * CS2;
      out[i] = WT[i] * s * (-1.0 + 0.5 * contraction * INV_CS2);
    }
  }
  // Sec. 2.3.2, eq. Siu.
  R s_i(int i, R vx, R vy) const {
    R cu = CX[i] * vx + CY[i] * vy;
    R uu = vx * vx + vy * vy;
    return WT[i] * (cu * INV_CS2 + 0.5 * cu * cu * INV_CS2 * INV_CS2 - 0.5 * uu * INV_CS2);
  }
  // Sec. 2.3.2, eq. G_i.
  void geq(R pp, R rh, R vx, R vy, R* out) const {
    for (int i = 0; i < Q; ++i)
      out[i] = (i == 0 ? pp * INV_CS2 * (WT[0] - 1.0) : pp * INV_CS2 * WT[i]) + rh * s_i(i, vx, vy);
  }
  // Sec. 2.3.2, eq. GGi (reading of the unbalanced parenthesis: the third
  // term is the dyad u grad(rho) contracted with c_i c_i - c_s^2 I, over c_s^2),
  // times the prefactor k: 1 - 1/(2 tau_g) for BGK, 1 for MRT (which applies
  // its prefactor per moment).
  void forcing(R k, R vx, R vy, R fx, R fy, R rx, R ry, R* out) const {
    R ugr = vx * rx + vy * ry;
    for (int i = 0; i < Q; ++i) {
      R cF = CX[i] * fx + CY[i] * fy;
      // (u grad rho) : (c c - c_s^2 I) = sum_ab u_a d_b rho (c_a c_b - c_s^2 delta_ab)
      R dyad = vx * rx * (CX[i] * CX[i] - CS2) + vx * ry * (CX[i] * CY[i]) +
               vy * rx * (CY[i] * CX[i]) + vy * ry * (CY[i] * CY[i] - CS2);
      out[i] = k * WT[i] * (ugr + cF * INV_CS2 + dyad * INV_CS2);
    }
  }
  // MRT: out_i = sum_k Minv[i][k] (rate_k m_k + pre_k n_k) with m = M a and
  // n = M b, i.e. the relaxation of a (rates) plus the forcing b (prefactors).
  static void mrt_apply(const R* rate, const R* pre, const R* a, const R* b, R* out) {
    R mk[Q];
    for (int k = 0; k < Q; ++k) {
      R ma = 0.0, mb = 0.0;
      for (int i = 0; i < Q; ++i) {
        ma += MB.M[k][i] * a[i];
        mb += MB.M[k][i] * b[i];
      }
      mk[k] = rate[k] * ma + pre[k] * mb;
    }
    for (int i = 0; i < Q; ++i) {
      R v = 0.0;
      for (int k = 0; k < Q; ++k) v += MB.M[k][i] / MB.norm2[k] * mk[k];
      out[i] = v;
    }
  }
  // Sec. 2.3.2, macroscopic subequations: u and p from g, rho, F, grad(rho).
  void macro(const R* gi, R rh, R fx, R fy, R rx, R ry, R& vx, R& vy, R& pp) const {
    R mx = 0.0, my = 0.0, sum_nz = 0.0;
    for (int i = 0; i < Q; ++i) {
      mx += CX[i] * gi[i];
      my += CY[i] * gi[i];
      if (i != 0) sum_nz += gi[i];
    }
    vx = (mx + 0.5 * fx) / rh;
    vy = (my + 0.5 * fy) / rh;
    pp = CS2 / (1.0 - WT[0]) * (sum_nz + 0.5 * (vx * rx + vy * ry) + rh * s_i(0, vx, vy));
  }

  // Steps 1-8 on the current pre-collision state.
  void compute_macro() {
    const size_t n = cells();
#pragma omp parallel for schedule(static)
    for (long k = 0; k < (long)n; ++k) {
      R s = 0.0;
      for (int i = 0; i < Q; ++i) s += f[i * n + k];
      phi[k] = s;
      rho[k] = density(s);
      nu[k] = viscosity(s);
    }
    chemical_potential(phi, mu);
    gradient(phi, gphx, gphy);
    gradient(mu, gmux, gmuy);
    gradient(rho, grhx, grhy);
#pragma omp parallel for schedule(static)
    for (long k = 0; k < (long)n; ++k) {
      Fx[k] = -phi[k] * gmux[k] + p.gx;
      Fy[k] = -phi[k] * gmuy[k] + p.gy;
      R gi[Q];
      for (int i = 0; i < Q; ++i) gi[i] = g[i * n + k];
      macro(gi, rho[k], Fx[k], Fy[k], grhx[k], grhy[k], ux[k], uy[k], pr[k]);
      S[k] = ux[k] * gphx[k] + uy[k] * gphy[k];
    }
  }

  // Steps 9-10.
  void collide() {
    const size_t n = cells();
#pragma omp parallel for schedule(static)
    for (long k = 0; k < (long)n; ++k) {
      R eq[Q], Fn[Q], Fo[Q], ge[Q], Gi[Q];
      const R omega_f = 1.0 / th.tau_f;  // eq. BGK multiplies the non-equilibrium part by 1/tau_f
      feq(phi[k], mu[k], eq);
      source(S[k], Fn);
      source(Sp[k], Fo);
      R tau_g = 0.5 + nu[k] * INV_CS2;  // viscosity-relaxation relation, solved for tau_g
      R omega_g = 1.0 / tau_g;
      geq(pr[k], rho[k], ux[k], uy[k], ge);
      if (p.collision == ORC_BGK) {
        for (int i = 0; i < Q; ++i) {
          R fi = f[i * n + k];
          // eq. BGK with delta_t = 1 and dF/dt ~ F(t) - F(t-1)
          fs[i * n + k] = fi - omega_f * (fi - eq[i]) + Fn[i] + 0.5 * (Fn[i] - Fo[i]);
        }
        forcing(1.0 - 1.0 / (2.0 * tau_g), ux[k], uy[k], Fx[k], Fy[k], grhx[k], grhy[k], Gi);
        for (int i = 0; i < Q; ++i) {
          R gi = g[i * n + k];
          gs[i * n + k] = gi - omega_g * (gi - ge[i]) + Gi[i];  // eq. BGK-NS
        }
      } else if (p.collision == ORC_MRT) {
        // moment order: rho, e, eps, j_x, q_x, j_y, q_y, p_xx, p_xy
        const R rf[Q] = {omega_f, p.mrt_f[0], p.mrt_f[1], omega_f, p.mrt_f[2],
                         omega_f, p.mrt_f[2], p.mrt_f[3], p.mrt_f[3]};
        const R rg[Q] = {p.mrt_g[0], p.mrt_g[0], p.mrt_g[0], omega_g, p.mrt_g[1],
                         omega_g, p.mrt_g[1], omega_g, omega_g};
        R zero[Q], pre_f[Q], pre_g[Q], df[Q], dg[Q], rel[Q];
        for (int q = 0; q < Q; ++q) {
          zero[q] = 0.0;
          pre_f[q] = 0.0;
          pre_g[q] = 1.0 - 0.5 * rg[q];
          df[q] = eq[q] - f[q * n + k];
          dg[q] = ge[q] - g[q * n + k];
        }
        mrt_apply(rf, pre_f, df, zero, rel);
        for (int i = 0; i < Q; ++i)
          fs[i * n + k] = f[i * n + k] + rel[i] + Fn[i] + 0.5 * (Fn[i] - Fo[i]);
        forcing(R(1.0), ux[k], uy[k], Fx[k], Fy[k], grhx[k], grhy[k], Gi);
        mrt_apply(rg, pre_g, dg, Gi, rel);
        for (int i = 0; i < Q; ++i) gs[i * n + k] = g[i * n + k] + rel[i];
      } else {
        std::abort();
      }
    }
  }

  // Step 11: f_i(x + c_i, t+1) = f*_i(x, t); a link that crosses a wall
  // returns to its own cell in the opposite direction.
  void stream() {
    const size_t n = cells();
    for (int i = 0; i < Q; ++i) {
      const int o = opposite(i);
#pragma omp parallel for schedule(static)
      for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
          int xx = x + CX[i], yy = y + CY[i];
          bool solid = (p.bc_x == ORC_WALL && (xx < 0 || xx >= nx)) ||
                       (p.bc_y == ORC_WALL && (yy < 0 || yy >= ny));
          size_t src = i * n + at(x, y);
          if (solid) {
            f[o * n + at(x, y)] = fs[src];
            g[o * n + at(x, y)] = gs[src];
          } else {
            size_t dst = i * n + at(((xx % nx) + nx) % nx, ((yy % ny) + ny) % ny);
            f[dst] = fs[src];
            g[dst] = gs[src];
          }
        }
    }
  }

  void step() {
    compute_macro();
    collide();
    stream();
    Sp = S;  // step 12
  }

  void init(const R* phi0, const R* u0x, const R* u0y) {
    const size_t n = cells();
    std::vector<R> ph(phi0, phi0 + n), m(n);
    chemical_potential(ph, m);
    for (size_t k = 0; k < n; ++k) {
      R eq[Q], ge[Q];
      feq(ph[k], m[k], eq);
      R vx = u0x ? u0x[k] : R(0.0), vy = u0y ? u0y[k] : R(0.0);
      geq(R(0.0), density(ph[k]), vx, vy, ge);
      for (int i = 0; i < Q; ++i) {
        f[i * n + k] = eq[i];
        g[i * n + k] = ge[i];
      }
    }
    compute_macro();
    Sp = S;
  }
};

template <class R>
Sim<R>* sim_of(void* h) { return static_cast<Sim<R>*>(h); }

template <class T>
void copy_out(const std::vector<T>& v, double* dst) {
  if (dst)
    for (size_t k = 0; k < v.size(); ++k) dst[k] = val(v[k]);
}

}  // namespace

extern "C" {

// ------------------------------------------------------------ lattice tables
void orc_lattice(int32_t* cx, int32_t* cy, double* w, double* cs2) {
  for (int i = 0; i < Q; ++i) { cx[i] = CX[i]; cy[i] = CY[i]; w[i] = WT[i]; }
  *cs2 = CS2;
}

void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}
int orc_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// -------------------------------------------------------- local definitions
// Single-cell forms, exposed so their moments can be checked against the
// moment identities the paper states (Sec. 2.3.1, eq. sumfeqandF).
void orc_feq(const orc_params* p, double phi, double mu, double* out) {
  Sim<double> s(*p); s.feq(phi, mu, out);
}
void orc_source(const orc_params* p, double S, double* out) {
  Sim<double> s(*p); s.source(S, out);
}
void orc_geq(const orc_params* p, double pr, double rho, double ux, double uy, double* out) {
  Sim<double> s(*p); s.geq(pr, rho, ux, uy, out);
}
void orc_forcing(const orc_params* p, double tau, double ux, double uy, double Fx, double Fy,
                 double rx, double ry, double* out) {
  Sim<double> s(*p); s.forcing(1.0 - 1.0 / (2.0 * tau), ux, uy, Fx, Fy, rx, ry, out);
}
void orc_macro(const orc_params* p, const double* g9, double rho, double Fx, double Fy,
               double rx, double ry, double* ux, double* uy, double* pr) {
  Sim<double> s(*p); s.macro(g9, rho, Fx, Fy, rx, ry, *ux, *uy, *pr);
}
// Discrete operators on a full field with the project's boundary rule.
void orc_gradient(const orc_params* p, const double* field, double* gx, double* gy) {
  Sim<double> s(*p);
  std::vector<double> v(field, field + s.cells()), ax(s.cells()), ay(s.cells());
  s.gradient(v, ax, ay);
  copy_out(ax, gx); copy_out(ay, gy);
}
void orc_laplacian(const orc_params* p, const double* field, double* out) {
  Sim<double> s(*p);
  std::vector<double> v(field, field + s.cells()), o(s.cells());
  s.laplacian(v, o);
  copy_out(o, out);
}
void orc_chemical_potential(const orc_params* p, const double* phi, double* out) {
  Sim<double> s(*p);
  std::vector<double> v(phi, phi + s.cells()), o(s.cells());
  s.chemical_potential(v, o);
  copy_out(o, out);
}
double orc_tau_f(const orc_params* p) { return 0.5 + p->M * INV_CS2 / p->alpha; }

// ------------------------------------------------------------- simulation
void* orc_create(const orc_params* p) { return new Sim<double>(*p); }
void orc_destroy(void* h) { delete sim_of<double>(h); }
void orc_init(void* h, const double* phi0, const double* u0x, const double* u0y) {
  sim_of<double>(h)->init(phi0, u0x, u0y);
}
void orc_step(void* h, int64_t n) {
  for (int64_t k = 0; k < n; ++k) sim_of<double>(h)->step();
}
// Moments of the current pre-collision state (steps 1-8, no collision).
void orc_moments(void* h, double* phi, double* mu, double* ux, double* uy, double* pr,
                 double* rho, double* S) {
  Sim<double>* s = sim_of<double>(h);
  s->compute_macro();
  copy_out(s->phi, phi); copy_out(s->mu, mu); copy_out(s->ux, ux); copy_out(s->uy, uy);
  copy_out(s->pr, pr); copy_out(s->rho, rho); copy_out(s->S, S);
}
void orc_get_state(void* h, double* f, double* g, double* Sp) {
  Sim<double>* s = sim_of<double>(h);
  copy_out(s->f, f); copy_out(s->g, g); copy_out(s->Sp, Sp);
}
void orc_set_state(void* h, const double* f, const double* g, const double* Sp) {
  Sim<double>* s = sim_of<double>(h);
  const size_t n = s->cells();
  for (size_t k = 0; k < Q * n; ++k) { s->f[k] = f[k]; s->g[k] = g[k]; }
  for (size_t k = 0; k < n; ++k) s->Sp[k] = Sp[k];
}

// ------------------------------------------------ tangent-linear model (TLM)
// dtheta = (d kappa, d beta, d alpha, d tau_f, d nu_A, d nu_B).
void* orc_tlm_create(const orc_params* p, const double* dtheta) {
  Sim<Dual>* s = new Sim<Dual>(*p);
  if (dtheta) {
    s->th.kappa.d = dtheta[0];
    s->th.beta.d = dtheta[1];
    s->th.alpha.d = dtheta[2];
    s->th.tau_f.d = dtheta[3];
    s->th.nu_A.d = dtheta[4];
    s->th.nu_B.d = dtheta[5];
  }
  return s;
}
void orc_tlm_destroy(void* h) { delete sim_of<Dual>(h); }
void orc_tlm_init(void* h, const double* phi0, const double* dphi0) {
  Sim<Dual>* s = sim_of<Dual>(h);
  const size_t n = s->cells();
  std::vector<Dual> ph(n);
  for (size_t k = 0; k < n; ++k) ph[k] = Dual(phi0[k], dphi0 ? dphi0[k] : 0.0);
  s->init(ph.data(), nullptr, nullptr);
}
void orc_tlm_set_state(void* h, const double* f, const double* df, const double* g,
                       const double* dg, const double* Sp, const double* dSp) {
  Sim<Dual>* s = sim_of<Dual>(h);
  const size_t n = s->cells();
  for (size_t k = 0; k < Q * n; ++k) {
    s->f[k] = Dual(f[k], df ? df[k] : 0.0);
    s->g[k] = Dual(g[k], dg ? dg[k] : 0.0);
  }
  for (size_t k = 0; k < n; ++k) s->Sp[k] = Dual(Sp[k], dSp ? dSp[k] : 0.0);
}
void orc_tlm_step(void* h, int64_t n) {
  for (int64_t k = 0; k < n; ++k) sim_of<Dual>(h)->step();
}
void orc_tlm_get_state(void* h, double* f, double* df, double* g, double* dg, double* Sp,
                       double* dSp) {
  Sim<Dual>* s = sim_of<Dual>(h);
  for (size_t k = 0; k < s->f.size(); ++k) {
    if (f) f[k] = s->f[k].v;
    if (df) df[k] = s->f[k].d;
    if (g) g[k] = s->g[k].v;
    if (dg) dg[k] = s->g[k].d;
  }
  for (size_t k = 0; k < s->Sp.size(); ++k) {
    if (Sp) Sp[k] = s->Sp[k].v;
    if (dSp) dSp[k] = s->Sp[k].d;
  }
}
// Tangent of the order parameter of the current state (phi = sum_i f_i).
void orc_tlm_phi(void* h, double* phi, double* dphi) {
  Sim<Dual>* s = sim_of<Dual>(h);
  const size_t n = s->cells();
  for (size_t k = 0; k < n; ++k) {
    Dual a = 0.0;
    for (int i = 0; i < Q; ++i) a += s->f[i * n + k];
    if (phi) phi[k] = a.v;
    if (dphi) dphi[k] = a.d;
  }
}

}  // extern "C"
