// WENO-ZN reference oracle -- TEST INFRASTRUCTURE ONLY.
//
// Plain, serial-by-construction, slow CPU implementation of the finite-difference
// WENO-ZN scheme of Shen, Zhang, Li and Peng, "A novel method for constructing high
// accurate and robust WENO-Z type scheme" (arXiv 2004.07954).  It exists so that the
// HIP library can be checked against something written directly from the paper.
// Only tests, the smoke check and the CPU-baseline leg of the benchmark may load it;
// the product path never does.  It shares no code with the HIP library.
//
// Everything is templated on the scalar type T:
//   double              -- the reference precision of all parity checks;
//   __float128          -- for the paper's critical-point table, whose errors fall
//                          below fp64 resolution;
//   std::complex<double>-- complex-step directional derivatives for the reference
//                          gradient of the discrete adjoint.
// Formulas are evaluated in the literal order the paper prints them, and the file is
// compiled with -ffp-contract=off so that no fused multiply-add changes that order.
// OpenMP pragmas only split independent per-cell loops; the max reduction is exact,
// so results do not depend on the thread count.
//
// Readings taken where the paper is silent (each is listed with its evidence in the
// design notes):
//   * eps of WENO-ZN is a parameter; 1e-40 reproduces the critical-point table.
//   * the exponent on tau8/(IS_k+eps) is a parameter q (paper: 1); the exponent on
//     the ratio inside C is p_C (paper: 2).
//   * tau inside C is tau5 = |IS0 - IS2|.
//   * f^- is reconstructed with the five points mirrored about x_{i+1/2}.
//   * Lax-Friedrichs alpha is the max of |u|+c over interior cells, recomputed for
//     every right-hand-side evaluation unless a frozen value is supplied.
//   * transmissive boundaries copy the edge cell into the three ghost cells.
//   * TVD-RK3 is the Shu-Osher three-stage scheme; dt comes from U^n.

#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>
#include <algorithm>
#include <quadmath.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef __float128 f128;
typedef std::complex<double> cplx;

// ---------------------------------------------------------------- scalar helpers
static inline double absv(double x) { return std::fabs(x); }
static inline f128 absv(f128 x) { return fabsq(x); }
// |z| for the complex step: the analytic continuation of |x| away from x = 0; at x = 0 the
// derivative is taken as 0 (the kink of tau5 = |IS0 - IS2| at symmetric stencils).
static inline cplx absv(cplx z) {
  if (z.real() > 0.0) return z;
  if (z.real() < 0.0) return -z;
  return cplx(0.0, 0.0);
}

static inline double sqrtv(double x) { return std::sqrt(x); }

static inline double realv(double x) { return x; }
static inline double realv(f128 x) { return (double)x; }
static inline double realv(cplx z) { return z.real(); }

template <class T> static inline T sq(T x) { return x * x; }
template <class T> static inline T ipow(T x, int p) {
  T r = x;
  for (int i = 1; i < p; ++i) r = r * x;
  return r;
}

// Scheme selector.  Only WZN_ZN is the paper's method; Z and JS are the comparison
// weights the paper restates (Sec. 2.1 eq:5, Sec. 2.2 eq:15), kept here only to check
// the test harness against the WENO-Z column of the critical-point table and as a
// negative control for the convergence-order tests.
enum { ORC_ZN = 0, ORC_Z = 1, ORC_JS = 2 };

struct OrcParams {       // mirrored by a ctypes Structure in oracle/binding.py
  int32_t scheme;        // ORC_ZN / ORC_Z / ORC_JS
  int32_t p_C;           // exponent in C (eq:function): 2
  int32_t q;             // exponent on tau/(IS_k+eps): ZN 1 (eq:new), Z q of eq:15
  int32_t pad;
  double A;              // constant of eq:function: 10
  double eps;            // epsilon
};

template <class T> struct Recon {
  T IS[3], tau5, tau8, C, alpha[3], omega[3], q[3], fhat;
};

// One fifth-order reconstruction of f_{i+1/2} from (f_{i-2}, ..., f_{i+2}) = (a..e).
//   candidate fluxes            Sec. 2.1, eq:4
//   Jiang-Shu indicators IS_k   Sec. 2.1, eq:isjiang
//   tau5 = |IS0 - IS2|          Sec. 2.2, eq:tao5 and Sec. 3, eq:tau
//   tau8                        Sec. 3, eq:tau8
//   C                           Sec. 3, eq:function
//   alpha_k (WENO-ZN)           Sec. 3, eq:new
//   omega_k, f_hat              Sec. 2.1, eq:5 and eq:3, with c = (0.1, 0.6, 0.3)
template <class T>
static Recon<T> reconstruct(T a, T b, T c, T d, T e, const OrcParams& P) {
  Recon<T> r;
  const T eps = T(P.eps);
  const T A = T(P.A);
  const T ck[3] = {T(1) / T(10), T(6) / T(10), T(3) / T(10)};

  r.q[0] = T(1) / T(3) * a - T(7) / T(6) * b + T(11) / T(6) * c;
  r.q[1] = -T(1) / T(6) * b + T(5) / T(6) * c + T(1) / T(3) * d;
  r.q[2] = T(1) / T(3) * c + T(5) / T(6) * d - T(1) / T(6) * e;

  r.IS[0] = T(13) / T(12) * sq(a - T(2) * b + c) + T(1) / T(4) * sq(a - T(4) * b + T(3) * c);
  r.IS[1] = T(13) / T(12) * sq(b - T(2) * c + d) + T(1) / T(4) * sq(b - d);
  // IS2 is written as the mirror image of IS0 (the same expression read from the other end
  // of the stencil), so that a stencil symmetric about x_i gives IS0 == IS2 exactly in
  // floating point, as it does in exact arithmetic.  Otherwise tau5 = |IS0 - IS2| is pure
  // rounding noise there and, with eps = 1e-40, C falls by tens of orders of magnitude.
  r.IS[2] = T(13) / T(12) * sq(e - T(2) * d + c) + T(1) / T(4) * sq(e - T(4) * d + T(3) * c);

  r.tau5 = absv(r.IS[0] - r.IS[2]);
  r.tau8 = sq(a - T(4) * b + T(6) * c - T(4) * d + e);
  r.C = A * ipow((r.IS[0] + r.IS[2] - r.tau5 + eps) / (r.tau5 + eps), P.p_C);

  for (int k = 0; k < 3; ++k) {
    if (P.scheme == ORC_ZN)
      r.alpha[k] = ck[k] * (r.C + ipow(r.tau8 / (r.IS[k] + eps), P.q));
    else if (P.scheme == ORC_Z)
      r.alpha[k] = ck[k] * (T(1) + ipow(r.tau5 / (r.IS[k] + eps), P.q));
    else
      r.alpha[k] = ck[k] / sq(r.IS[k] + eps);
  }
  const T sum = r.alpha[0] + r.alpha[1] + r.alpha[2];
  for (int k = 0; k < 3; ++k) r.omega[k] = r.alpha[k] / sum;
  r.fhat = r.omega[0] * r.q[0] + r.omega[1] * r.q[1] + r.omega[2] * r.q[2];
  return r;
}

// ---------------------------------------------------------------- physics
// Systems: 0 = linear advection u_t + a u_x = 0 (Sec. 4.2, eq:26);
//          1 = 1D Euler, U = (rho, rho u, E) (Sec. 4.3);
//          2 = 2D Euler, U = (rho, rho u, rho v, E) (Sec. 4.4, eq:2d).
enum { SYS_ADV = 0, SYS_EULER1 = 1, SYS_EULER2 = 2 };
enum { BC_PERIODIC = 0, BC_TRANSMISSIVE = 1 };

struct Phys {
  double a;      // advection speed
  double gamma;  // ratio of specific heats
};

// 1D Euler: u = m/rho; p from E = p/(gamma-1) + rho u^2 / 2; F = (rho u, rho u^2 + p, u (E + p)).
template <class T>
static void euler1_flux(const T* U, T* F, const Phys& ph) {
  const T rho = U[0], m = U[1], E = U[2];
  const T u = m / rho;
  const T p = (T(ph.gamma) - T(1)) * (E - T(1) / T(2) * rho * u * u);
  F[0] = rho * u;
  F[1] = rho * u * u + p;
  F[2] = u * (E + p);
}

static double euler1_speed(const double* U, const Phys& ph) {
  const double rho = U[0], m = U[1], E = U[2];
  const double u = m / rho;
  const double p = (ph.gamma - 1.0) * (E - 0.5 * rho * u * u);
  return std::fabs(u) + std::sqrt(ph.gamma * p / rho);
}

// 2D Euler, E = p/(gamma-1) + rho (u^2 + v^2)/2;
// F = (rho u, rho u^2 + p, rho u v, u (E + p)), G = (rho v, rho u v, rho v^2 + p, v (E + p)).
template <class T>
static void euler2_flux(const T* U, T* F, T* G, const Phys& ph) {
  const T rho = U[0], mx = U[1], my = U[2], E = U[3];
  const T u = mx / rho, v = my / rho;
  const T p = (T(ph.gamma) - T(1)) * (E - rho / T(2) * (u * u + v * v));
  F[0] = rho * u; F[1] = rho * u * u + p; F[2] = rho * u * v; F[3] = u * (E + p);
  G[0] = rho * v; G[1] = rho * u * v; G[2] = rho * v * v + p; G[3] = v * (E + p);
}

static void euler2_speeds(const double* U, const Phys& ph, double* sx, double* sy) {
  const double rho = U[0], mx = U[1], my = U[2], E = U[3];
  const double u = mx / rho, v = my / rho;
  const double p = (ph.gamma - 1.0) * (E - rho / 2.0 * (u * u + v * v));
  const double c = std::sqrt(ph.gamma * p / rho);
  *sx = std::fabs(u) + c;
  *sy = std::fabs(v) + c;
}

// Steger-Warming flux-vector splitting of the 2D Euler flux along the unit direction
// (nx, ny) = (1, 0) for F or (0, 1) for G (Sec. 4.4 cites it; the ideal-gas form).  With the
// normal velocity un, the eigenvalues l = (un - c, un, un, un + c) and l^{+-} = (l +- |l|)/2,
//   F^{+-} = rho/(2 gamma) * ( 2(gamma-1) l2 + l1 + l4,
//                              2(gamma-1) l2 u + l1 (u - c nx) + l4 (u + c nx),
//                              2(gamma-1) l2 v + l1 (v - c ny) + l4 (v + c ny),
//                              (gamma-1) l2 (u^2 + v^2) + l1/2 ((u - c nx)^2 + (v - c ny)^2)
//                                + l4/2 ((u + c nx)^2 + (v + c ny)^2)
//                                + (3 - gamma)(l1 + l4) c^2 / (2 (gamma - 1)) ).
// No entropy fix: |l| is used as it is.  F^+ + F^- = F (exactly, in exact arithmetic).
template <class T>
static void sw_split(const T* U, int dir, int sign, T* Fs, const Phys& ph) {
  const T g = T(ph.gamma);
  const T rho = U[0], u = U[1] / rho, v = U[2] / rho;
  const T p = (g - T(1)) * (U[3] - rho / T(2) * (u * u + v * v));
  const T c = sqrtv(g * p / rho);
  const T nx = dir == 0 ? T(1) : T(0), ny = dir == 0 ? T(0) : T(1);
  const T un = dir == 0 ? u : v;
  const T s = sign > 0 ? T(1) : T(-1);
  const T l1 = (un - c + s * absv(un - c)) / T(2);
  const T l2 = (un + s * absv(un)) / T(2);
  const T l4 = (un + c + s * absv(un + c)) / T(2);
  const T k = rho / (T(2) * g);
  const T um = u - c * nx, vm = v - c * ny, up = u + c * nx, vp = v + c * ny;
  Fs[0] = k * (T(2) * (g - T(1)) * l2 + l1 + l4);
  Fs[1] = k * (T(2) * (g - T(1)) * l2 * u + l1 * um + l4 * up);
  Fs[2] = k * (T(2) * (g - T(1)) * l2 * v + l1 * vm + l4 * vp);
  Fs[3] = k * ((g - T(1)) * l2 * (u * u + v * v) + l1 / T(2) * (um * um + vm * vm) +
               l4 / T(2) * (up * up + vp * vp) +
               (T(3) - g) * (l1 + l4) * c * c / (T(2) * (g - T(1))));
}

static int nvar_of(int sys) { return sys == SYS_ADV ? 1 : (sys == SYS_EULER1 ? 3 : 4); }

// Ghost index map for three ghost cells per side (Sec. 4.2, eq:26 periodic; the
// transmissive rule copies the edge cell).
static inline int64_t ghost_index(int64_t g, int64_t n, int bc) {
  if (g >= 0 && g < n) return g;
  if (bc == BC_PERIODIC) return ((g % n) + n) % n;
  return g < 0 ? 0 : n - 1;
}

// ---------------------------------------------------------------- 1D right-hand side
// Global Lax-Friedrichs alpha for the 1D systems: max over interior cells of the
// largest wave speed (Sec. 4.3: |u| + c with c = sqrt(gamma p / rho); advection: |a|).
static double lf_alpha_1d(int sys, int64_t n, const double* u, const Phys& ph) {
  if (sys == SYS_ADV) return std::fabs(ph.a);
  double m = 0.0;
#pragma omp parallel for reduction(max : m)
  for (int64_t i = 0; i < n; ++i) {
    double U[3] = {u[i], u[n + i], u[2 * n + i]};
    m = std::max(m, euler1_speed(U, ph));
  }
  return m;
}

// L_i = -(fhat_{i+1/2} - fhat_{i-1/2}) / dx (Sec. 2, eq:2), with
// fhat = fhat^+ + fhat^-, fhat^+ from (f+_{i-2..i+2}) and fhat^- from the mirrored
// (f-_{i+3}, ..., f-_{i-1}) (the symmetric rule about x_{i+1/2}, Sec. 2), and the
// Lax-Friedrichs split f^{+-} = (F(U) +- alpha U)/2 applied component by component.
template <class T>
static void rhs_1d(int sys, int bc, int64_t n, const T* u, T* dudt, T dx, double alpha,
                   const OrcParams& P, const Phys& ph) {
  const int nv = nvar_of(sys);
  const int64_t np = n + 6;  // padded: cell i lives at i + 3
  std::vector<T> Up(nv * np), fp(nv * np), fm(nv * np), fh(nv * (n + 1));
  for (int v = 0; v < nv; ++v)
    for (int64_t g = -3; g < n + 3; ++g) Up[v * np + g + 3] = u[v * n + ghost_index(g, n, bc)];

#pragma omp parallel for
  for (int64_t j = 0; j < np; ++j) {
    T U[3], F[3];
    for (int v = 0; v < nv; ++v) U[v] = Up[v * np + j];
    if (sys == SYS_ADV) F[0] = T(ph.a) * U[0];
    else euler1_flux(U, F, ph);
    for (int v = 0; v < nv; ++v) {
      fp[v * np + j] = T(1) / T(2) * (F[v] + T(alpha) * U[v]);
      fm[v * np + j] = T(1) / T(2) * (F[v] - T(alpha) * U[v]);
    }
  }
  // interface k <-> x_{i+1/2} with i = k - 1, k = 0..n
#pragma omp parallel for
  for (int64_t k = 0; k <= n; ++k) {
    const int64_t i = k - 1 + 3;  // padded index of cell i
    for (int v = 0; v < nv; ++v) {
      const T* P_ = &fp[v * np];
      const T* M_ = &fm[v * np];
      T hp = reconstruct(P_[i - 2], P_[i - 1], P_[i], P_[i + 1], P_[i + 2], P).fhat;
      T hm = reconstruct(M_[i + 3], M_[i + 2], M_[i + 1], M_[i], M_[i - 1], P).fhat;
      fh[v * (n + 1) + k] = hp + hm;
    }
  }
  for (int v = 0; v < nv; ++v)
    for (int64_t i = 0; i < n; ++i)
      dudt[v * n + i] = -(fh[v * (n + 1) + i + 1] - fh[v * (n + 1) + i]) / dx;
}

// ---------------------------------------------------------------- 1D Euler, local characteristic fields
// Sec. 4.3: Lax-Friedrichs splitting with the WENO reconstruction carried out in local
// characteristic fields (the procedure of the scheme family the paper cites there).  The paper
// gives no further detail; the readings taken are:
//   * the state at x_{i+1/2} is the Roe average of U_i and U_{i+1}
//     (u, H = (E + p)/rho weighted by sqrt(rho); c^2 = (gamma - 1)(H - u^2/2));
//   * R has the right eigenvectors of the flux Jacobian there as columns,
//     (1, u - c, H - u c), (1, u, u^2/2), (1, u + c, H + u c), and Lc = R^{-1};
//   * the split is made field by field: g+-_j = (Lc F_j +- alpha_k Lc U_j)/2 over the stencil
//     cells, alpha_k = max over interior cells of |lambda_k(U_j)|, lambda = (u - c, u, u + c),
//     recomputed per RHS evaluation;
//   * ghat_k = WZN(g+_{i-2..i+2}) + WZN(g-_{i+3..i-1}) (mirrored), fhat = R ghat.
template <class T>
static void roe_eigen(const T* UL, const T* UR, const Phys& ph, T R[3][3], T Lc[3][3]) {
  const T g = T(ph.gamma);
  const T uL = UL[1] / UL[0], uR = UR[1] / UR[0];
  const T pL = (g - T(1)) * (UL[2] - T(1) / T(2) * UL[0] * uL * uL);
  const T pR = (g - T(1)) * (UR[2] - T(1) / T(2) * UR[0] * uR * uR);
  const T HL = (UL[2] + pL) / UL[0], HR = (UR[2] + pR) / UR[0];
  const T sL = sqrtv(UL[0]), sR = sqrtv(UR[0]);
  const T u = (sL * uL + sR * uR) / (sL + sR);
  const T H = (sL * HL + sR * HR) / (sL + sR);
  const T c = sqrtv((g - T(1)) * (H - T(1) / T(2) * u * u));
  R[0][0] = T(1);          R[0][1] = T(1);                R[0][2] = T(1);
  R[1][0] = u - c;         R[1][1] = u;                   R[1][2] = u + c;
  R[2][0] = H - u * c;     R[2][1] = T(1) / T(2) * u * u; R[2][2] = H + u * c;
  const T b1 = (g - T(1)) / (c * c);
  const T b2 = T(1) / T(2) * u * u * b1;
  Lc[0][0] = T(1) / T(2) * (b2 + u / c);
  Lc[0][1] = -T(1) / T(2) * (b1 * u + T(1) / c);
  Lc[0][2] = T(1) / T(2) * b1;
  Lc[1][0] = T(1) - b2;
  Lc[1][1] = b1 * u;
  Lc[1][2] = -b1;
  Lc[2][0] = T(1) / T(2) * (b2 - u / c);
  Lc[2][1] = -T(1) / T(2) * (b1 * u - T(1) / c);
  Lc[2][2] = T(1) / T(2) * b1;
}

// Per-field global LF alphas: max over interior cells of |u - c|, |u|, |u + c|.
static void lf_alpha_char(int64_t n, const double* u, const Phys& ph, double* a3) {
  double m0 = 0.0, m1 = 0.0, m2 = 0.0;
#pragma omp parallel for reduction(max : m0, m1, m2)
  for (int64_t i = 0; i < n; ++i) {
    const double rho = u[i], m = u[n + i], E = u[2 * n + i];
    const double v = m / rho;
    const double p = (ph.gamma - 1.0) * (E - 0.5 * rho * v * v);
    const double c = std::sqrt(ph.gamma * p / rho);
    m0 = std::max(m0, std::fabs(v - c));
    m1 = std::max(m1, std::fabs(v));
    m2 = std::max(m2, std::fabs(v + c));
  }
  a3[0] = m0; a3[1] = m1; a3[2] = m2;
}

template <class T>
static void rhs_1d_char(int bc, int64_t n, const T* u, T* dudt, T dx, const double* a3,
                        const OrcParams& P, const Phys& ph) {
  const int64_t np = n + 6;  // padded: cell i lives at i + 3
  std::vector<T> Up(3 * np), Fp(3 * np), fh(3 * (n + 1));
  for (int v = 0; v < 3; ++v)
    for (int64_t g = -3; g < n + 3; ++g) Up[v * np + g + 3] = u[v * n + ghost_index(g, n, bc)];
  for (int64_t j = 0; j < np; ++j) {
    T U[3] = {Up[j], Up[np + j], Up[2 * np + j]}, F[3];
    euler1_flux(U, F, ph);
    for (int v = 0; v < 3; ++v) Fp[v * np + j] = F[v];
  }
#pragma omp parallel for
  for (int64_t k = 0; k <= n; ++k) {
    const int64_t i = k - 1 + 3;  // padded index of cell i; interface x_{i+1/2}
    T UL[3] = {Up[i], Up[np + i], Up[2 * np + i]};
    T UR[3] = {Up[i + 1], Up[np + i + 1], Up[2 * np + i + 1]};
    T R[3][3], Lc[3][3];
    roe_eigen(UL, UR, ph, R, Lc);
    // characteristic split fluxes over the cells i-2 .. i+3
    T gp[3][6], gm[3][6];
    for (int j = 0; j < 6; ++j) {
      const int64_t cj = i - 2 + j;
      for (int f = 0; f < 3; ++f) {
        T V = T(0), G = T(0);
        for (int v = 0; v < 3; ++v) {
          V = V + Lc[f][v] * Up[v * np + cj];
          G = G + Lc[f][v] * Fp[v * np + cj];
        }
        gp[f][j] = T(1) / T(2) * (G + T(a3[f]) * V);
        gm[f][j] = T(1) / T(2) * (G - T(a3[f]) * V);
      }
    }
    T gh[3];
    for (int f = 0; f < 3; ++f) {
      // positions 0..5 <-> cells i-2 .. i+3
      T hp = reconstruct(gp[f][0], gp[f][1], gp[f][2], gp[f][3], gp[f][4], P).fhat;
      T hm = reconstruct(gm[f][5], gm[f][4], gm[f][3], gm[f][2], gm[f][1], P).fhat;
      gh[f] = hp + hm;
    }
    for (int v = 0; v < 3; ++v) {
      T s = T(0);
      for (int f = 0; f < 3; ++f) s = s + R[v][f] * gh[f];
      fh[v * (n + 1) + k] = s;
    }
  }
  for (int v = 0; v < 3; ++v)
    for (int64_t i = 0; i < n; ++i)
      dudt[v * n + i] = -(fh[v * (n + 1) + i + 1] - fh[v * (n + 1) + i]) / dx;
}

// ---------------------------------------------------------------- 2D right-hand side
// Dimension by dimension (Sec. 4.4, eq:2d): L = -(Fhat_{i+1/2,j} - Fhat_{i-1/2,j})/dx
// - (Ghat_{i,j+1/2} - Ghat_{i,j-1/2})/dy, each a 1D WENO-ZN reconstruction of the split
// flux along its own direction: Lax-Friedrichs with its own global alpha (split = 0), or the
// Steger-Warming splitting the paper uses for its 2D problems (split = 1; the alphas are not
// used).  Layout [4][ny][nx], x fastest.
enum { SPLIT_LF = 0, SPLIT_SW = 1 };
template <class T>
static void rhs_2d(int bcx, int bcy, int64_t nx, int64_t ny, const T* u, T* dudt, T dx, T dy,
                   double ax, double ay, const OrcParams& P, const Phys& ph, int split = SPLIT_LF) {
  const int64_t N = nx * ny;
#pragma omp parallel for
  for (int64_t j = 0; j < ny; ++j) {
    // x sweep along row j
    const int64_t np = nx + 6;
    std::vector<T> fp(4 * np), fm(4 * np), fh(4 * (nx + 1));
    for (int64_t g = -3; g < nx + 3; ++g) {
      const int64_t gi = ghost_index(g, nx, bcx);
      T U[4], F[4], G[4], Sp[4], Sm[4];
      for (int v = 0; v < 4; ++v) U[v] = u[v * N + j * nx + gi];
      euler2_flux(U, F, G, ph);
      if (split == SPLIT_SW) { sw_split(U, 0, +1, Sp, ph); sw_split(U, 0, -1, Sm, ph); }
      for (int v = 0; v < 4; ++v) {
        fp[v * np + g + 3] = split == SPLIT_SW ? Sp[v] : T(1) / T(2) * (F[v] + T(ax) * U[v]);
        fm[v * np + g + 3] = split == SPLIT_SW ? Sm[v] : T(1) / T(2) * (F[v] - T(ax) * U[v]);
      }
    }
    for (int64_t k = 0; k <= nx; ++k) {
      const int64_t i = k - 1 + 3;
      for (int v = 0; v < 4; ++v) {
        const T* P_ = &fp[v * np];
        const T* M_ = &fm[v * np];
        fh[v * (nx + 1) + k] =
            reconstruct(P_[i - 2], P_[i - 1], P_[i], P_[i + 1], P_[i + 2], P).fhat +
            reconstruct(M_[i + 3], M_[i + 2], M_[i + 1], M_[i], M_[i - 1], P).fhat;
      }
    }
    for (int v = 0; v < 4; ++v)
      for (int64_t i = 0; i < nx; ++i)
        dudt[v * N + j * nx + i] = -(fh[v * (nx + 1) + i + 1] - fh[v * (nx + 1) + i]) / dx;
  }
#pragma omp parallel for
  for (int64_t i = 0; i < nx; ++i) {
    // y sweep along column i
    const int64_t np = ny + 6;
    std::vector<T> gp(4 * np), gm(4 * np), gh(4 * (ny + 1));
    for (int64_t g = -3; g < ny + 3; ++g) {
      const int64_t gj = ghost_index(g, ny, bcy);
      T U[4], F[4], G[4], Sp[4], Sm[4];
      for (int v = 0; v < 4; ++v) U[v] = u[v * N + gj * nx + i];
      euler2_flux(U, F, G, ph);
      if (split == SPLIT_SW) { sw_split(U, 1, +1, Sp, ph); sw_split(U, 1, -1, Sm, ph); }
      for (int v = 0; v < 4; ++v) {
        gp[v * np + g + 3] = split == SPLIT_SW ? Sp[v] : T(1) / T(2) * (G[v] + T(ay) * U[v]);
        gm[v * np + g + 3] = split == SPLIT_SW ? Sm[v] : T(1) / T(2) * (G[v] - T(ay) * U[v]);
      }
    }
    for (int64_t k = 0; k <= ny; ++k) {
      const int64_t jj = k - 1 + 3;
      for (int v = 0; v < 4; ++v) {
        const T* P_ = &gp[v * np];
        const T* M_ = &gm[v * np];
        gh[v * (ny + 1) + k] =
            reconstruct(P_[jj - 2], P_[jj - 1], P_[jj], P_[jj + 1], P_[jj + 2], P).fhat +
            reconstruct(M_[jj + 3], M_[jj + 2], M_[jj + 1], M_[jj], M_[jj - 1], P).fhat;
      }
    }
    for (int v = 0; v < 4; ++v)
      for (int64_t j = 0; j < ny; ++j)
        dudt[v * N + j * nx + i] += -(gh[v * (ny + 1) + j + 1] - gh[v * (ny + 1) + j]) / dy;
  }
}

static void lf_alpha_2d(int64_t N, const double* u, const Phys& ph, double* ax, double* ay) {
  double mx = 0.0, my = 0.0;
#pragma omp parallel for reduction(max : mx, my)
  for (int64_t k = 0; k < N; ++k) {
    double U[4] = {u[k], u[N + k], u[2 * N + k], u[3 * N + k]};
    double sx, sy;
    euler2_speeds(U, ph, &sx, &sy);
    mx = std::max(mx, sx);
    my = std::max(my, sy);
  }
  *ax = mx;
  *ay = my;
}

// ---------------------------------------------------------------- 2D Euler, local characteristic fields
// The 1D procedure of Sec. 4.3 applied along each sweep direction n = (nx, ny) of the
// dimension-by-dimension scheme (eq:2d): (1, 0) for the x sweep, (0, 1) for the y sweep.  At
// x_{i+1/2} (or y_{j+1/2}) the flux Jacobian A_n = nx dF/dU + ny dG/dU is taken at the Roe
// average of the two neighbouring states (u, v and H = (E + p)/rho weighted by sqrt(rho),
// c^2 = (gamma - 1)(H - (u^2 + v^2)/2)), with u_n = u nx + v ny, u_t = -u ny + v nx.  Its
// eigenvalues are u_n - c, u_n, u_n, u_n + c; R has the right eigenvectors as columns,
//   (1, u - c nx, v - c ny, H - c u_n), (1, u, v, q^2/2), (0, -ny, nx, u_t),
//   (1, u + c nx, v + c ny, H + c u_n),
// and Lc = R^{-1}.  The split, the per-field alphas (max over interior cells of |lambda_k| of
// the cell states, per sweep and per RHS evaluation) and ghat = WZN(g+) + WZN(g-) mirrored
// follow the 1D procedure; the interface flux is R ghat.
template <class T>
static void roe_eigen_2d(const T* UL, const T* UR, int dir, const Phys& ph, T R[4][4],
                         T Lc[4][4]) {
  const T g = T(ph.gamma);
  const T nx = dir == 0 ? T(1) : T(0), ny = dir == 0 ? T(0) : T(1);
  const T uL = UL[1] / UL[0], vL = UL[2] / UL[0];
  const T uR = UR[1] / UR[0], vR = UR[2] / UR[0];
  const T pL = (g - T(1)) * (UL[3] - T(1) / T(2) * UL[0] * (uL * uL + vL * vL));
  const T pR = (g - T(1)) * (UR[3] - T(1) / T(2) * UR[0] * (uR * uR + vR * vR));
  const T HL = (UL[3] + pL) / UL[0], HR = (UR[3] + pR) / UR[0];
  const T sL = sqrtv(UL[0]), sR = sqrtv(UR[0]);
  const T u = (sL * uL + sR * uR) / (sL + sR);
  const T v = (sL * vL + sR * vR) / (sL + sR);
  const T H = (sL * HL + sR * HR) / (sL + sR);
  const T q2 = u * u + v * v;
  const T c = sqrtv((g - T(1)) * (H - T(1) / T(2) * q2));
  const T un = u * nx + v * ny, ut = -u * ny + v * nx;
  const T col[4][4] = {{T(1), u - c * nx, v - c * ny, H - c * un},
                       {T(1), u, v, T(1) / T(2) * q2},
                       {T(0), -ny, nx, ut},
                       {T(1), u + c * nx, v + c * ny, H + c * un}};
  for (int r = 0; r < 4; ++r)
    for (int f = 0; f < 4; ++f) R[r][f] = col[f][r];
  const T b1 = (g - T(1)) / (c * c);
  const T b2 = T(1) / T(2) * q2 * b1;
  Lc[0][0] = T(1) / T(2) * (b2 + un / c);
  Lc[0][1] = -T(1) / T(2) * (b1 * u + nx / c);
  Lc[0][2] = -T(1) / T(2) * (b1 * v + ny / c);
  Lc[0][3] = T(1) / T(2) * b1;
  Lc[1][0] = T(1) - b2;
  Lc[1][1] = b1 * u;
  Lc[1][2] = b1 * v;
  Lc[1][3] = -b1;
  Lc[2][0] = -ut;
  Lc[2][1] = -ny;
  Lc[2][2] = nx;
  Lc[2][3] = T(0);
  Lc[3][0] = T(1) / T(2) * (b2 - un / c);
  Lc[3][1] = -T(1) / T(2) * (b1 * u - nx / c);
  Lc[3][2] = -T(1) / T(2) * (b1 * v - ny / c);
  Lc[3][3] = T(1) / T(2) * b1;
}

// Per-field global alphas of a 2D state: x sweep max |u - c|, |u|, |u|, |u + c| (a[0..3]),
// y sweep max |v - c|, |v|, |v|, |v + c| (a[4..7]).
static void lf_alpha_2d_char(int64_t N, const double* u, const Phys& ph, double* a8) {
  double m0 = 0, m1 = 0, m2 = 0, m3 = 0, m4 = 0, m5 = 0;
#pragma omp parallel for reduction(max : m0, m1, m2, m3, m4, m5)
  for (int64_t k = 0; k < N; ++k) {
    const double rho = u[k], mx = u[N + k], my = u[2 * N + k], E = u[3 * N + k];
    const double uu = mx / rho, vv = my / rho;
    const double p = (ph.gamma - 1.0) * (E - rho / 2.0 * (uu * uu + vv * vv));
    const double c = std::sqrt(ph.gamma * p / rho);
    m0 = std::max(m0, std::fabs(uu - c));
    m1 = std::max(m1, std::fabs(uu));
    m2 = std::max(m2, std::fabs(uu + c));
    m3 = std::max(m3, std::fabs(vv - c));
    m4 = std::max(m4, std::fabs(vv));
    m5 = std::max(m5, std::fabs(vv + c));
  }
  a8[0] = m0; a8[1] = m1; a8[2] = m1; a8[3] = m2;
  a8[4] = m3; a8[5] = m4; a8[6] = m4; a8[7] = m5;
}

// One characteristic sweep along a line of n cells (stride `st` in the state arrays, plane N):
// adds -(fhat_{i+1/2} - fhat_{i-1/2}) / h to dudt along the line.
template <class T>
static void char_sweep_2d(int bc, int dir, int64_t n, int64_t base, int64_t st, int64_t N,
                          const T* u, T* dudt, T h, const double* a4, const OrcParams& P,
                          const Phys& ph) {
  const int64_t np = n + 6;
  std::vector<T> Up(4 * np), Fp(4 * np), fh(4 * (n + 1));
  for (int64_t g = -3; g < n + 3; ++g) {
    const int64_t gi = ghost_index(g, n, bc);
    T U[4], F[4], G[4];
    for (int v = 0; v < 4; ++v) U[v] = u[v * N + base + gi * st];
    euler2_flux(U, F, G, ph);
    for (int v = 0; v < 4; ++v) {
      Up[v * np + g + 3] = U[v];
      Fp[v * np + g + 3] = dir == 0 ? F[v] : G[v];
    }
  }
  for (int64_t k = 0; k <= n; ++k) {
    const int64_t i = k - 1 + 3;
    T UL[4], UR[4];
    for (int v = 0; v < 4; ++v) { UL[v] = Up[v * np + i]; UR[v] = Up[v * np + i + 1]; }
    T R[4][4], Lc[4][4];
    roe_eigen_2d(UL, UR, dir, ph, R, Lc);
    T gp[4][6], gm[4][6];
    for (int j = 0; j < 6; ++j) {
      const int64_t cj = i - 2 + j;
      for (int f = 0; f < 4; ++f) {
        T V = T(0), G = T(0);
        for (int v = 0; v < 4; ++v) {
          V = V + Lc[f][v] * Up[v * np + cj];
          G = G + Lc[f][v] * Fp[v * np + cj];
        }
        gp[f][j] = T(1) / T(2) * (G + T(a4[f]) * V);
        gm[f][j] = T(1) / T(2) * (G - T(a4[f]) * V);
      }
    }
    T gh[4];
    for (int f = 0; f < 4; ++f) {
      T hp = reconstruct(gp[f][0], gp[f][1], gp[f][2], gp[f][3], gp[f][4], P).fhat;
      T hm = reconstruct(gm[f][5], gm[f][4], gm[f][3], gm[f][2], gm[f][1], P).fhat;
      gh[f] = hp + hm;
    }
    for (int v = 0; v < 4; ++v) {
      T s = T(0);
      for (int f = 0; f < 4; ++f) s = s + R[v][f] * gh[f];
      fh[v * (n + 1) + k] = s;
    }
  }
  for (int v = 0; v < 4; ++v)
    for (int64_t i = 0; i < n; ++i)
      dudt[v * N + base + i * st] += -(fh[v * (n + 1) + i + 1] - fh[v * (n + 1) + i]) / h;
}

template <class T>
static void rhs_2d_char(int bcx, int bcy, int64_t nx, int64_t ny, const T* u, T* dudt, T dx,
                        T dy, const double* a8, const OrcParams& P, const Phys& ph) {
  const int64_t N = nx * ny;
  for (int64_t k = 0; k < 4 * N; ++k) dudt[k] = T(0);
#pragma omp parallel for
  for (int64_t j = 0; j < ny; ++j)
    char_sweep_2d<T>(bcx, 0, nx, j * nx, 1, N, u, dudt, dx, a8, P, ph);
#pragma omp parallel for
  for (int64_t i = 0; i < nx; ++i)
    char_sweep_2d<T>(bcy, 1, ny, i, nx, N, u, dudt, dy, a8 + 4, P, ph);
}

// ---------------------------------------------------------------- TVD-RK3
// Shu-Osher third-order TVD Runge-Kutta (cited in Sec. 4; standard form):
//   U1 = U^n + dt L(U^n)
//   U2 = 3/4 U^n + 1/4 (U1 + dt L(U1))
//   U^{n+1} = 1/3 U^n + 2/3 (U2 + dt L(U2))
static const double RK_A[3] = {0.0, 3.0 / 4.0, 1.0 / 3.0};
static const double RK_B[3] = {1.0, 1.0 / 4.0, 2.0 / 3.0};

extern "C" {

typedef struct {
  double alpha_used[3];  // LF alpha of each stage (x direction)
  double alpha_used_y[3];
  double dt;
} OrcStepInfo;

// ---- single reconstruction, all intermediate quantities (fp64)
// out: IS0 IS1 IS2 tau5 tau8 C alpha0..2 omega0..2 q0..2 fhat  (16 doubles)
void orc_reconstruct_f64(const double* f5, const OrcParams* P, double* out) {
  Recon<double> r = reconstruct(f5[0], f5[1], f5[2], f5[3], f5[4], *P);
  double* o = out;
  for (int k = 0; k < 3; ++k) *o++ = r.IS[k];
  *o++ = r.tau5; *o++ = r.tau8; *o++ = r.C;
  for (int k = 0; k < 3; ++k) *o++ = r.alpha[k];
  for (int k = 0; k < 3; ++k) *o++ = r.omega[k];
  for (int k = 0; k < 3; ++k) *o++ = r.q[k];
  *o++ = r.fhat;
}

// Same in __float128; inputs/outputs as (hi, lo) pairs of doubles, value = hi + lo.
void orc_reconstruct_f128(const double* f5hi, const double* f5lo, const OrcParams* P,
                          double* out_hi, double* out_lo) {
  f128 f[5];
  for (int k = 0; k < 5; ++k) f[k] = (f128)f5hi[k] + (f128)f5lo[k];
  Recon<f128> r = reconstruct(f[0], f[1], f[2], f[3], f[4], *P);
  f128 vals[16];
  f128* o = vals;
  for (int k = 0; k < 3; ++k) *o++ = r.IS[k];
  *o++ = r.tau5; *o++ = r.tau8; *o++ = r.C;
  for (int k = 0; k < 3; ++k) *o++ = r.alpha[k];
  for (int k = 0; k < 3; ++k) *o++ = r.omega[k];
  for (int k = 0; k < 3; ++k) *o++ = r.q[k];
  *o++ = r.fhat;
  for (int k = 0; k < 16; ++k) {
    out_hi[k] = (double)vals[k];
    out_lo[k] = (double)(vals[k] - (f128)out_hi[k]);
  }
}

// ---- 1D RHS (fp64).  alpha_in < 0: compute the global LF alpha from u.
double orc_rhs_1d_f64(int sys, int bc, int64_t n, const double* u, double* dudt, double dx,
                      double alpha_in, const OrcParams* P, double a, double gamma) {
  Phys ph{a, gamma};
  double alpha = alpha_in >= 0.0 ? alpha_in : lf_alpha_1d(sys, n, u, ph);
  rhs_1d<double>(sys, bc, n, u, dudt, dx, alpha, *P, ph);
  return alpha;
}

// ---- 1D RHS in __float128 (hi/lo pairs); alpha must be supplied.
void orc_rhs_1d_f128(int sys, int bc, int64_t n, const double* uhi, const double* ulo,
                     double* dhi, double* dlo, double dx_hi, double dx_lo, double alpha,
                     const OrcParams* P, double a, double gamma) {
  Phys ph{a, gamma};
  const int nv = nvar_of(sys);
  std::vector<f128> u(nv * n), d(nv * n);
  for (int64_t k = 0; k < nv * n; ++k) u[k] = (f128)uhi[k] + (f128)ulo[k];
  rhs_1d<f128>(sys, bc, n, u.data(), d.data(), (f128)dx_hi + (f128)dx_lo, alpha, *P, ph);
  for (int64_t k = 0; k < nv * n; ++k) {
    dhi[k] = (double)d[k];
    dlo[k] = (double)(d[k] - (f128)dhi[k]);
  }
}

// ---- 1D RHS with complex inputs (complex-step derivatives); alpha must be supplied.
// Arrays are interleaved (re, im) pairs.
void orc_rhs_1d_c128(int sys, int bc, int64_t n, const double* u_ri, double* d_ri, double dx,
                     double alpha, const OrcParams* P, double a, double gamma) {
  Phys ph{a, gamma};
  const int nv = nvar_of(sys);
  std::vector<cplx> u(nv * n), d(nv * n);
  for (int64_t k = 0; k < nv * n; ++k) u[k] = cplx(u_ri[2 * k], u_ri[2 * k + 1]);
  rhs_1d<cplx>(sys, bc, n, u.data(), d.data(), cplx(dx, 0.0), alpha, *P, ph);
  for (int64_t k = 0; k < nv * n; ++k) {
    d_ri[2 * k] = d[k].real();
    d_ri[2 * k + 1] = d[k].imag();
  }
}

// ---- one TVD-RK3 step, 1D (fp64), in place on u.
// dt_in <= 0: dt = cfl dx / max(|u|+c) of U^n (Sec. 4.3); advection uses |a|.
// alpha_in: NULL -> LF alpha recomputed for every stage from that stage's input;
//           otherwise alpha_in[s] is the frozen alpha of stage s.
void orc_rk3_step_1d_f64(int sys, int bc, int64_t n, double* u, double dx, double cfl,
                         double dt_in, const double* alpha_in, const OrcParams* P, double a,
                         double gamma, OrcStepInfo* info) {
  Phys ph{a, gamma};
  const int nv = nvar_of(sys);
  const int64_t M = nv * n;
  std::vector<double> un(u, u + M), us(u, u + M), L(M);
  const double speed = lf_alpha_1d(sys, n, u, ph);
  const double dt = dt_in > 0.0 ? dt_in : cfl * dx / speed;
  for (int s = 0; s < 3; ++s) {
    const double alpha = alpha_in ? alpha_in[s] : lf_alpha_1d(sys, n, us.data(), ph);
    rhs_1d<double>(sys, bc, n, us.data(), L.data(), dx, alpha, *P, ph);
    for (int64_t k = 0; k < M; ++k)
      us[k] = RK_A[s] * un[k] + RK_B[s] * (us[k] + dt * L[k]);
    if (info) info->alpha_used[s] = alpha;
  }
  std::memcpy(u, us.data(), sizeof(double) * M);
  if (info) info->dt = dt;
}

// ---- nsteps TVD-RK3 steps, 1D.  dt_in: NULL (CFL) or [nsteps];
// alpha_in: NULL (reduce) or [3*nsteps]; dt_out/alpha_out may be NULL.
void orc_rk3_run_1d_f64(int sys, int bc, int64_t n, double* u, double dx, double cfl,
                        int32_t nsteps, const double* dt_in, const double* alpha_in,
                        const OrcParams* P, double a, double gamma, double* dt_out,
                        double* alpha_out) {
  for (int32_t s = 0; s < nsteps; ++s) {
    OrcStepInfo info;
    orc_rk3_step_1d_f64(sys, bc, n, u, dx, cfl, dt_in ? dt_in[s] : -1.0,
                        alpha_in ? alpha_in + 3 * s : nullptr, P, a, gamma, &info);
    if (dt_out) dt_out[s] = info.dt;
    if (alpha_out)
      for (int k = 0; k < 3; ++k) alpha_out[3 * s + k] = info.alpha_used[k];
  }
}

// ---- one TVD-RK3 step with complex state (complex-step derivatives of the step map),
// dt and the three stage alphas frozen.  u_ri: interleaved (re, im), updated in place.
void orc_rk3_step_1d_c128(int sys, int bc, int64_t n, double* u_ri, double dx, double dt,
                          const double* alpha3, const OrcParams* P, double a, double gamma) {
  Phys ph{a, gamma};
  const int nv = nvar_of(sys);
  const int64_t M = nv * n;
  std::vector<cplx> un(M), us(M), L(M);
  for (int64_t k = 0; k < M; ++k) un[k] = us[k] = cplx(u_ri[2 * k], u_ri[2 * k + 1]);
  for (int s = 0; s < 3; ++s) {
    rhs_1d<cplx>(sys, bc, n, us.data(), L.data(), cplx(dx, 0.0), alpha3[s], *P, ph);
    for (int64_t k = 0; k < M; ++k)
      us[k] = cplx(RK_A[s]) * un[k] + cplx(RK_B[s]) * (us[k] + cplx(dt) * L[k]);
  }
  for (int64_t k = 0; k < M; ++k) {
    u_ri[2 * k] = us[k].real();
    u_ri[2 * k + 1] = us[k].imag();
  }
}

// ---- nsteps TVD-RK3 steps with complex state and the frozen schedule dts[nsteps],
// alphas[nsteps][3] (complex-step directional derivatives of a whole run): the step above,
// applied nsteps times.  u_ri: interleaved (re, im), updated in place.
void orc_rk3_run_1d_c128(int sys, int bc, int64_t n, double* u_ri, double dx, int32_t nsteps,
                         const double* dts, const double* alphas, const OrcParams* P, double a,
                         double gamma) {
  for (int32_t s = 0; s < nsteps; ++s)
    orc_rk3_step_1d_c128(sys, bc, n, u_ri, dx, dts[s], alphas + 3 * s, P, a, gamma);
}

// ---- nsteps TVD-RK3 steps in __float128 with the frozen schedule dts[nsteps],
// alphas[nsteps][3] (reference values of a whole run below fp64 resolution, e.g. finite
// differences with steps far below the fp64 spacing of the state).  The state is carried in
// __float128 between steps; input and output as (hi, lo) pairs, value = hi + lo.
void orc_rk3_run_1d_f128(int sys, int bc, int64_t n, double* uhi, double* ulo, double dx,
                         int32_t nsteps, const double* dts, const double* alphas,
                         const OrcParams* P, double a, double gamma) {
  Phys ph{a, gamma};
  const int nv = nvar_of(sys);
  const int64_t M = nv * n;
  std::vector<f128> un(M), us(M), L(M);
  for (int64_t k = 0; k < M; ++k) un[k] = (f128)uhi[k] + (f128)ulo[k];
  const f128 rk_a[3] = {f128(0), f128(3) / f128(4), f128(1) / f128(3)};
  const f128 rk_b[3] = {f128(1), f128(1) / f128(4), f128(2) / f128(3)};
  for (int32_t st = 0; st < nsteps; ++st) {
    us = un;
    const f128 dt = (f128)dts[st];
    for (int s = 0; s < 3; ++s) {
      rhs_1d<f128>(sys, bc, n, us.data(), L.data(), (f128)dx, alphas[3 * st + s], *P, ph);
      for (int64_t k = 0; k < M; ++k) us[k] = rk_a[s] * un[k] + rk_b[s] * (us[k] + dt * L[k]);
    }
    un = us;
  }
  for (int64_t k = 0; k < M; ++k) {
    uhi[k] = (double)un[k];
    ulo[k] = (double)(un[k] - (f128)uhi[k]);
  }
}

// ---- 2D RHS (fp64).  alpha_x/alpha_y < 0: compute from u.  Returns both alphas.
void orc_rhs_2d_f64(int bcx, int bcy, int64_t nx, int64_t ny, const double* u, double* dudt,
                    double dx, double dy, double alpha_x, double alpha_y, const OrcParams* P,
                    double gamma, double* alpha_used) {
  Phys ph{0.0, gamma};
  double ax, ay;
  lf_alpha_2d(nx * ny, u, ph, &ax, &ay);
  if (alpha_x >= 0.0) ax = alpha_x;
  if (alpha_y >= 0.0) ay = alpha_y;
  rhs_2d<double>(bcx, bcy, nx, ny, u, dudt, dx, dy, ax, ay, *P, ph);
  if (alpha_used) { alpha_used[0] = ax; alpha_used[1] = ay; }
}

// ---- nsteps TVD-RK3 steps, 2D, in place.  dt from U^n as
// dt = cfl dtx dty / (dtx + dty), dtx = dx / max(|u|+c), dty = dy / max(|v|+c)
// (Sec. 4.4).  LF alphas recomputed for every stage.
void orc_rk3_run_2d_f64(int bcx, int bcy, int64_t nx, int64_t ny, double* u, double dx,
                        double dy, double cfl, int32_t nsteps, const double* dt_in,
                        const OrcParams* P, double gamma, double* dt_out) {
  Phys ph{0.0, gamma};
  const int64_t M = 4 * nx * ny;
  std::vector<double> un(M), us(M), L(M);
  for (int32_t st = 0; st < nsteps; ++st) {
    std::memcpy(un.data(), u, sizeof(double) * M);
    std::memcpy(us.data(), u, sizeof(double) * M);
    double sx, sy;
    lf_alpha_2d(nx * ny, u, ph, &sx, &sy);
    const double dtx = dx / sx, dty = dy / sy;
    const double dt = dt_in ? dt_in[st] : cfl * dtx * dty / (dtx + dty);
    for (int s = 0; s < 3; ++s) {
      double ax, ay;
      lf_alpha_2d(nx * ny, us.data(), ph, &ax, &ay);
      rhs_2d<double>(bcx, bcy, nx, ny, us.data(), L.data(), dx, dy, ax, ay, *P, ph);
      for (int64_t k = 0; k < M; ++k)
        us[k] = RK_A[s] * un[k] + RK_B[s] * (us[k] + dt * L[k]);
    }
    std::memcpy(u, us.data(), sizeof(double) * M);
    if (dt_out) dt_out[st] = dt;
  }
}

// ---- 2D RHS with the Steger-Warming splitting (fp64).
void orc_rhs_2d_sw_f64(int bcx, int bcy, int64_t nx, int64_t ny, const double* u, double* dudt,
                       double dx, double dy, const OrcParams* P, double gamma) {
  Phys ph{0.0, gamma};
  rhs_2d<double>(bcx, bcy, nx, ny, u, dudt, dx, dy, 0.0, 0.0, *P, ph, SPLIT_SW);
}

// ---- Steger-Warming split fluxes of one 2D state along dir (0: x, 1: y): Fp, Fm [4].
void orc_sw_split_f64(const double* U, int dir, double gamma, double* Fp, double* Fm) {
  Phys ph{0.0, gamma};
  sw_split<double>(U, dir, +1, Fp, ph);
  sw_split<double>(U, dir, -1, Fm, ph);
}

// ---- nsteps TVD-RK3 steps, 2D, Steger-Warming splitting, in place; dt as in
// orc_rk3_run_2d_f64 (Sec. 4.4).
void orc_rk3_run_2d_sw_f64(int bcx, int bcy, int64_t nx, int64_t ny, double* u, double dx,
                           double dy, double cfl, int32_t nsteps, const double* dt_in,
                           const OrcParams* P, double gamma, double* dt_out) {
  Phys ph{0.0, gamma};
  const int64_t M = 4 * nx * ny;
  std::vector<double> un(M), us(M), L(M);
  for (int32_t st = 0; st < nsteps; ++st) {
    std::memcpy(un.data(), u, sizeof(double) * M);
    std::memcpy(us.data(), u, sizeof(double) * M);
    double sx, sy;
    lf_alpha_2d(nx * ny, u, ph, &sx, &sy);
    const double dtx = dx / sx, dty = dy / sy;
    const double dt = dt_in ? dt_in[st] : cfl * dtx * dty / (dtx + dty);
    for (int s = 0; s < 3; ++s) {
      rhs_2d<double>(bcx, bcy, nx, ny, us.data(), L.data(), dx, dy, 0.0, 0.0, *P, ph, SPLIT_SW);
      for (int64_t k = 0; k < M; ++k)
        us[k] = RK_A[s] * un[k] + RK_B[s] * (us[k] + dt * L[k]);
    }
    std::memcpy(u, us.data(), sizeof(double) * M);
    if (dt_out) dt_out[st] = dt;
  }
}

// ---- 1D Euler in local characteristic fields (fp64).  alpha3_in: NULL -> the per-field
// global alphas of u; otherwise the three frozen alphas.  alpha3_out (may be NULL) receives the
// alphas used.
void orc_rhs_1d_char_f64(int bc, int64_t n, const double* u, double* dudt, double dx,
                         const double* alpha3_in, const OrcParams* P, double gamma,
                         double* alpha3_out) {
  Phys ph{0.0, gamma};
  double a3[3];
  if (alpha3_in) { a3[0] = alpha3_in[0]; a3[1] = alpha3_in[1]; a3[2] = alpha3_in[2]; }
  else lf_alpha_char(n, u, ph, a3);
  rhs_1d_char<double>(bc, n, u, dudt, dx, a3, *P, ph);
  if (alpha3_out) for (int f = 0; f < 3; ++f) alpha3_out[f] = a3[f];
}

// The eigenvector matrices at the Roe average of two states (row-major R then Lc).
void orc_roe_eigen_f64(const double* UL, const double* UR, double gamma, double* R9,
                       double* L9) {
  Phys ph{0.0, gamma};
  double R[3][3], Lc[3][3];
  roe_eigen(UL, UR, ph, R, Lc);
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) { R9[3 * r + c] = R[r][c]; L9[3 * r + c] = Lc[r][c]; }
}

// ---- nsteps TVD-RK3 steps of the characteristic scheme, in place.  dt from U^n as
// cfl dx / max(|u| + c) (Sec. 4.3) unless dt_in [nsteps] gives it; per-field alphas
// recomputed for every stage.  dt_out [nsteps] and alpha_out [nsteps][3 stages][3 fields] may
// be NULL.
void orc_rk3_run_1d_char_f64(int bc, int64_t n, double* u, double dx, double cfl,
                             int32_t nsteps, const double* dt_in, const OrcParams* P,
                             double gamma, double* dt_out, double* alpha_out) {
  Phys ph{0.0, gamma};
  const int64_t M = 3 * n;
  std::vector<double> un(M), us(M), L(M);
  for (int32_t st = 0; st < nsteps; ++st) {
    std::memcpy(un.data(), u, sizeof(double) * M);
    std::memcpy(us.data(), u, sizeof(double) * M);
    const double dt = dt_in ? dt_in[st] : cfl * dx / lf_alpha_1d(SYS_EULER1, n, u, ph);
    for (int s = 0; s < 3; ++s) {
      double a3[3];
      lf_alpha_char(n, us.data(), ph, a3);
      rhs_1d_char<double>(bc, n, us.data(), L.data(), dx, a3, *P, ph);
      for (int64_t k = 0; k < M; ++k)
        us[k] = RK_A[s] * un[k] + RK_B[s] * (us[k] + dt * L[k]);
      if (alpha_out) for (int f = 0; f < 3; ++f) alpha_out[9 * st + 3 * s + f] = a3[f];
    }
    std::memcpy(u, us.data(), sizeof(double) * M);
    if (dt_out) dt_out[st] = dt;
  }
}

// ---- 2D Euler in local characteristic fields (fp64).  alpha8_in: NULL -> the per-field
// global alphas of u (x sweep a[0..3], y sweep a[4..7]); alpha8_out (may be NULL) receives
// the alphas used.
void orc_rhs_2d_char_f64(int bcx, int bcy, int64_t nx, int64_t ny, const double* u,
                         double* dudt, double dx, double dy, const double* alpha8_in,
                         const OrcParams* P, double gamma, double* alpha8_out) {
  Phys ph{0.0, gamma};
  double a8[8];
  if (alpha8_in) for (int f = 0; f < 8; ++f) a8[f] = alpha8_in[f];
  else lf_alpha_2d_char(nx * ny, u, ph, a8);
  rhs_2d_char<double>(bcx, bcy, nx, ny, u, dudt, dx, dy, a8, *P, ph);
  if (alpha8_out) for (int f = 0; f < 8; ++f) alpha8_out[f] = a8[f];
}

// The 2D eigenvector matrices along dir (0: x, 1: y) at the Roe average (row-major R, Lc).
void orc_roe_eigen_2d_f64(const double* UL, const double* UR, int dir, double gamma,
                          double* R16, double* L16) {
  Phys ph{0.0, gamma};
  double R[4][4], Lc[4][4];
  roe_eigen_2d(UL, UR, dir, ph, R, Lc);
  for (int r = 0; r < 4; ++r)
    for (int c = 0; c < 4; ++c) { R16[4 * r + c] = R[r][c]; L16[4 * r + c] = Lc[r][c]; }
}

// ---- nsteps TVD-RK3 steps of the 2D characteristic scheme, in place; dt as in
// orc_rk3_run_2d_f64 (Sec. 4.4), per-field alphas recomputed for every stage.
void orc_rk3_run_2d_char_f64(int bcx, int bcy, int64_t nx, int64_t ny, double* u, double dx,
                             double dy, double cfl, int32_t nsteps, const double* dt_in,
                             const OrcParams* P, double gamma, double* dt_out) {
  Phys ph{0.0, gamma};
  const int64_t M = 4 * nx * ny;
  std::vector<double> un(M), us(M), L(M);
  for (int32_t st = 0; st < nsteps; ++st) {
    std::memcpy(un.data(), u, sizeof(double) * M);
    std::memcpy(us.data(), u, sizeof(double) * M);
    double sx, sy;
    lf_alpha_2d(nx * ny, u, ph, &sx, &sy);
    const double dtx = dx / sx, dty = dy / sy;
    const double dt = dt_in ? dt_in[st] : cfl * dtx * dty / (dtx + dty);
    for (int s = 0; s < 3; ++s) {
      double a8[8];
      lf_alpha_2d_char(nx * ny, us.data(), ph, a8);
      rhs_2d_char<double>(bcx, bcy, nx, ny, us.data(), L.data(), dx, dy, a8, *P, ph);
      for (int64_t k = 0; k < M; ++k)
        us[k] = RK_A[s] * un[k] + RK_B[s] * (us[k] + dt * L[k]);
    }
    std::memcpy(u, us.data(), sizeof(double) * M);
    if (dt_out) dt_out[st] = dt;
  }
}

// Thread count the OpenMP runtime would use (reported with CPU timings).
int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

// Set the thread count of the per-cell loops (results do not depend on it: the only
// reductions are exact maxima).
void orc_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

}  // extern "C"
