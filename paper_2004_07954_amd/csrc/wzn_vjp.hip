// Hand-written discrete adjoint of the 1D WENO-ZN right-hand side and of the TVD-RK3 step.
//
// The map differentiated is the one the forward kernels evaluate, with the Lax-Friedrichs
// alpha of every stage and the dt of every step frozen (they are recorded by the forward run
// and treated as constants).  For L_i = -(fhat_{i+1/2} - fhat_{i-1/2}) / dx (Sec. 2, eq:2) the
// cotangent of interface flux fhat_{e+1/2} is nu_e = (mu_{e+1} - mu_e) / dx; it is pulled back
// through the two reconstructions of that interface (f^+ stencil, and the f^- stencil
// mirrored about x_{e+1/2}), through the Lax-Friedrichs split f^{+-} = (F(U) +- alpha U)/2
// and the Euler flux Jacobian, and through the boundary index map (ghost cells add their
// cotangent to the cell they copy).
//
// One workgroup owns a run of interfaces, one per thread, and the cells between them.  It
// stages the split fluxes of the cells the interfaces read and the cotangents mu in LDS,
// computes per interface the ten scaled partial derivatives nu_e * d fhat_e / d f^{+-}(cell),
// and each output cell then gathers the partials of the (at most six) interfaces whose
// stencils contain it.
//
// Stage adjoint (fused): with v = mu + dt J(U_s)^T mu,
//   out = p v + q acc_in,   acc_out = r acc_in + s mu
// which covers the three stages of the TVD-RK3 adjoint recurrence
//   lam2 = 2/3 (lam3 + dt J2^T lam3),        acc = 1/3 lam3
//   lam1 = 1/4 (lam2 + dt J1^T lam2),        acc = acc + 3/4 lam2
//   lam0 = acc + lam1 + dt J0^T lam1.
#include <hip/hip_runtime.h>

#include "wzn_device.hpp"
#include "wzn_host.hpp"
#include "wzn_rows.hpp"
#include "wzn_tile.hpp"

namespace wzn {

struct VjpArgs {
  const double* U;       // stage state [3][n] at which L is linearised
  const double* mu;      // cotangent of L (or of the stage output) [3][n]
  const double* acc_in;  // [3][n] or null
  double* out;           // [3][n]
  double* acc_out;       // [3][n] or null; may alias acc_in (same element, same thread)
  int64_t n;
  double dx;
  int bc;
  double gamma, eps, A;
  const double* alpha_arr;  // frozen alpha (device) or null
  double alpha_const;
  const double* dt_arr;     // frozen dt (device) or null (plain VJP)
  int stage_mode;           // 0: out = J^T mu; 1: fused stage adjoint
  double p, q, r, s;
};

// 1/x from one v_rcp_f64 (relative error up to ~5e-8) and one Newton step (~2e-15): enough
// for a derivative that is compared at 1e-10.
__device__ __forceinline__ double rcp1(double x) {
  const double r = __builtin_amdgcn_rcp(x);
  return __builtin_fma(__builtin_fma(-x, r, 1.0), r, r);
}

// f-hat of one reconstruction (Sec. 2.1 eq:3-5, Sec. 3 eq:function, eq:tau8, eq:new) and
// g[k] = nu * d fhat / d v[k], evaluated in the paper's literal form (fp64 carries the
// magnitudes of C and tau8/(IS_k+eps) for eps = 1e-40).  d|x|/dx is taken as 0 at x = 0.
__device__ __forceinline__ void wzn_grad(const double* v, double nu, double eps, double A,
                                         double* g) {
  const double a = v[0], b = v[1], c = v[2], d = v[3], e = v[4];
  const double A0 = a - 2.0 * b + c, B0 = a - 4.0 * b + 3.0 * c;
  const double A1 = b - 2.0 * c + d, B1 = b - d;
  // IS2 as the mirror image of IS0 (the same expression read from e back to c), so that a
  // stencil symmetric about its centre gives IS0 == IS2, hence tau5 = 0, exactly in floating
  // point as in exact arithmetic: the forward kernels' difference form has this property, and
  // the linearisation must see the same tau5 (d|x|/dx at 0 is taken as 0)
  const double A2 = e - 2.0 * d + c, B2 = e - 4.0 * d + 3.0 * c;
  const double IS0 = (13.0 / 12.0) * A0 * A0 + 0.25 * B0 * B0;
  const double IS1 = (13.0 / 12.0) * A1 * A1 + 0.25 * B1 * B1;
  const double IS2 = (13.0 / 12.0) * A2 * A2 + 0.25 * B2 * B2;
  const double d4 = a - 4.0 * b + 6.0 * c - 4.0 * d + e;
  const double tau8 = d4 * d4;
  const double diff = IS0 - IS2;
  const double t5 = __builtin_fabs(diff);
  const double num = IS0 + IS2 - t5 + eps, den = t5 + eps;
  const double iden = rcp1(den);
  const double r = num * iden;
  const double C = A * r * r;
  const double ck[3] = {0.1, 0.6, 0.3};
  const double s[3] = {IS0 + eps, IS1 + eps, IS2 + eps};
  double is[3], t[3], al[3];
  double S = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    is[k] = rcp1(s[k]);
    t[k] = tau8 * is[k];
    al[k] = ck[k] * (C + t[k]);
    S += al[k];
  }
  const double iS = rcp1(S);
  // q_k - q_1 from second differences (eq:4): no cancellation of the O(f) parts
  const double dq[3] = {(A0 - A1) * (1.0 / 3.0), 0.0, (A1 - A2) * (1.0 / 6.0)};
  double tbar = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) tbar += ck[k] * t[k];
  double om[3], fr = 0.0;  // fr = fhat - q_1 = sum_k omega_k (q_k - q_1)
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    om[k] = al[k] * iS;
    fr += om[k] * dq[k];
  }
  // reverse sweep.  omega_k - c_k = c_k (t_k - tbar) / S is formed without the (possibly huge)
  // C, and sum_k c_k (q_k - fhat) = -sum_k (omega_k - c_k)(q_k - q_1): where C dominates,
  // both are tiny differences that a direct evaluation would bury in rounding noise, which
  // the 1/den of dC/dtau5 then amplifies.
  double Cb = 0.0, tau8b = 0.0, sb[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double wk = ck[k] * (t[k] - tbar) * iS;
    Cb -= nu * wk * dq[k] * iS;
    const double tb = ck[k] * nu * (dq[k] - fr) * iS;  // c_k * dL/dalpha_k
    tau8b += tb * is[k];
    sb[k] = -tb * t[k] * is[k];
  }
  const double rb = Cb * 2.0 * A * r;
  const double numb = rb * iden;
  const double denb = -rb * r * iden;
  double IS0b = sb[0] + numb, IS1b = sb[1], IS2b = sb[2] + numb;
  const double t5b = -numb + denb;
  const double sg = diff > 0.0 ? 1.0 : (diff < 0.0 ? -1.0 : 0.0);
  IS0b += sg * t5b;
  IS2b -= sg * t5b;
  const double d4b = 2.0 * d4 * tau8b;
  const double A0b = (13.0 / 6.0) * A0 * IS0b, B0b = 0.5 * B0 * IS0b;
  const double A1b = (13.0 / 6.0) * A1 * IS1b, B1b = 0.5 * B1 * IS1b;
  const double A2b = (13.0 / 6.0) * A2 * IS2b, B2b = 0.5 * B2 * IS2b;
  const double qb0 = nu * om[0], qb1 = nu * om[1], qb2 = nu * om[2];
  g[0] = d4b + A0b + B0b + qb0 * (1.0 / 3.0);
  g[1] = -4.0 * d4b - 2.0 * A0b - 4.0 * B0b + A1b + B1b - qb0 * (7.0 / 6.0) - qb1 * (1.0 / 6.0);
  g[2] = 6.0 * d4b + A0b + 3.0 * B0b - 2.0 * A1b + A2b + 3.0 * B2b + qb0 * (11.0 / 6.0) +
         qb1 * (5.0 / 6.0) + qb2 * (1.0 / 3.0);
  g[3] = -4.0 * d4b + A1b - B1b - 2.0 * A2b - 4.0 * B2b + qb1 * (1.0 / 3.0) + qb2 * (5.0 / 6.0);
  g[4] = d4b + A2b + B2b - qb2 * (1.0 / 6.0);
}

// Boundary index map: periodic wrap or transmissive clamp of any cell index p.  Indices
// within one period of the grid wrap by one addition; the 64-bit remainder (a long software
// sequence on the GPU) only runs further out, for rows shorter than a tile.
__device__ __forceinline__ int64_t map_cell(int64_t p, int64_t n, int bc) {
  if (p >= 0 && p < n) return p;
  if (bc != 0) return p < 0 ? 0 : n - 1;
  if (p < 0 && p >= -n) return p + n;
  if (p >= n && p < 2 * n) return p - n;
  p %= n;
  return p < 0 ? p + n : p;
}

// One workgroup owns VJP_NI interfaces, e = g0 - 3 + i (the right interface of cell e), and the
// VJP_NI - 5 cells g0 .. g0 + VJP_NI - 6 whose six interfaces (e = j - 3 .. j + 2) all lie among
// them; tiles overlap by five interfaces.  One thread per (sign, component, interface) pulls
// nu_e back through one reconstruction, so that the ~130 instructions of a reconstruction's
// reverse sweep are spread over six threads per interface (the kernel is short and
// latency-bound at the adjoint workload's size).  Every global load is issued at kernel start:
// the states of the cells the stencils read (g0 - 5 .. g0 + VJP_NI - 1), the cotangents mu of
// g0 - 3 .. g0 + VJP_NI - 3, and the accumulator of the output cells.
// 72 interfaces (432 threads, 67 output cells) with at most 72 VGPRs (7 waves per SIMD, 20 B
// of spills): four workgroups per CU, so the adjoint workload's 979 workgroups run in one
// round; 64 interfaces at 76 VGPRs took 1111 workgroups in two (backward pass 2 % slower).
constexpr int VJP_NI = 72;
constexpr int VJP_NT = 6 * VJP_NI;
constexpr int VJP_TC = VJP_NI - 5;  // output cells per workgroup

__global__ __launch_bounds__(VJP_NT) __attribute__((amdgpu_waves_per_eu(7)))
void vjp_kernel(VjpArgs a) {
  constexpr int NI = VJP_NI, TC = VJP_TC;
  constexpr int NW = NI + 5;  // staged cells g0 - 5 .. g0 + NI - 1
  constexpr int NM = NI + 1;  // staged cotangents g0 - 3 .. g0 + NI - 3
  __shared__ double Wp[3][NW], Wm[3][NW], US[3][NW], MU[3][NM], G[3][10][NI];
  const int tid = threadIdx.x;
  const int64_t n = a.n;
  const int64_t g0 = (int64_t)blockIdx.x * TC;
  const double alpha = a.alpha_arr ? a.alpha_arr[0] : a.alpha_const;
  const double gm1 = a.gamma - 1.0;

  // ---- loads: staged states (threads 0 .. NW-1), cotangents (threads 128 .. 128+NM-1),
  //      accumulator of the output cells (threads 256 .. 256+TC-1)
  double Uc[3], muv[3], accv[3];
  const int tm = tid - 128, ta = tid - 256;
  const int64_t jo = g0 + ta;  // output cell of threads 256 ..
  if (tid < NW) {
    const int64_t cell = map_cell(g0 - 5 + tid, n, a.bc);
#pragma unroll
    for (int c = 0; c < 3; ++c) Uc[c] = a.U[c * n + cell];
  } else if (tm >= 0 && tm < NM) {
    const int64_t cell = g0 - 3 + tm;
    int64_t src = -1;
    if (a.bc == 0) src = map_cell(cell, n, 0);
    else if (cell >= 0 && cell < n) src = cell;
#pragma unroll
    for (int c = 0; c < 3; ++c) muv[c] = src >= 0 ? a.mu[c * n + src] : 0.0;
  } else if (ta >= 0 && ta < TC && jo < n && a.stage_mode && a.acc_in) {
#pragma unroll
    for (int c = 0; c < 3; ++c) accv[c] = a.acc_in[c * n + jo];
  }
  if (tid < NW) {
    const double rho = Uc[0], m = Uc[1], E = Uc[2];
    const double u = m / rho;
    const double p = gm1 * (E - 0.5 * rho * u * u);
    const double F[3] = {rho * u, rho * u * u + p, u * (E + p)};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      Wp[c][tid] = 0.5 * (F[c] + alpha * Uc[c]);
      Wm[c][tid] = 0.5 * (F[c] - alpha * Uc[c]);
      US[c][tid] = Uc[c];
    }
  } else if (tm >= 0 && tm < NM) {
#pragma unroll
    for (int c = 0; c < 3; ++c) MU[c][tm] = muv[c];
  }
  __syncthreads();

  // ---- one reconstruction per thread: sign sg, component c, interface slot i.  G[c][k][i]
  //      holds nu_e d fhat^+_e / d f^+(cell e-2+k) (k = 0..4) and nu_e d fhat^-_e /
  //      d f^-(cell e+3-(k-5)) (k = 5..9)
  {
    const int sg = tid / (3 * NI), c = (tid / NI) % 3, i = tid % NI;
    const int64_t e = g0 - 3 + i;
    const bool valid = a.bc == 0 || (e >= -1 && e <= n - 1);
    const double nu = valid ? (MU[c][i + 1] - MU[c][i]) * (1.0 / a.dx) : 0.0;
    double v[5], g[5];
    if (sg == 0) {
#pragma unroll
      for (int k = 0; k < 5; ++k) v[k] = Wp[c][i + k];  // cells e-2 .. e+2
    } else {
#pragma unroll
      for (int k = 0; k < 5; ++k) v[k] = Wm[c][i + 5 - k];  // cells e+3 .. e-1
    }
    wzn_grad(v, nu, a.eps, a.A, g);
#pragma unroll
    for (int k = 0; k < 5; ++k) G[c][5 * sg + k][i] = g[k];
  }
  __syncthreads();

  // ---- output cells: gather, flux Jacobian, stage combination
  if (ta < 0 || ta >= TC || jo >= n) return;
  const int t = ta;
  const int64_t j = jo;
  const bool interior = j >= 5 && j + 5 < n;
  int64_t mc[11];
  if (!interior) {
#pragma unroll
    for (int q = 0; q < 11; ++q) mc[q] = map_cell(j - 5 + q, n, a.bc);
  }
  double wbp[3], wbm[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double sp = 0.0, sm = 0.0;
    if (interior) {
      // cell j is slot k of the f^+ stencil of interface j + 2 - k (slot t + 5 - k) and slot
      // 5 + k of the f^- stencil of interface j - 3 + k (slot t + k)
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        sp += G[c][k][t + 5 - k];
        sm += G[c][5 + k][t + k];
      }
    } else {
      // near the ends of the row: every stencil slot that the boundary index map sends to j
      // (stencil cells lie within j - 5 .. j + 5; mc[q] is the image of cell j - 5 + q)
#pragma unroll
      for (int de = -3; de <= 2; ++de) {
        const int slot = t + 3 + de;
#pragma unroll
        for (int k = 0; k < 5; ++k) {
          if (mc[de + k + 3] == j) sp += G[c][k][slot];      // cell j + de - 2 + k
          if (mc[de - k + 8] == j) sm += G[c][5 + k][slot];  // cell j + de + 3 - k
        }
      }
    }
    wbp[c] = sp;
    wbm[c] = sm;
  }

  // f^{+-}_c = (F_c +- alpha U_c)/2:  Ubar_d = 1/2 sum_c (wbp_c + wbm_c) dF_c/dU_d
  //                                          + alpha/2 (wbp_d - wbm_d)
  const double rho = US[0][t + 5], m = US[1][t + 5], E = US[2][t + 5];
  const double u = m / rho;
  const double p = gm1 * (E - 0.5 * rho * u * u);
  const double H = (E + p) / rho;
  // Jacobian of F = (m, m^2/rho + p, u (E + p)) with p = (gamma-1)(E - m^2/(2 rho))
  const double J[3][3] = {
      {0.0, 1.0, 0.0},
      {0.5 * (a.gamma - 3.0) * u * u, (3.0 - a.gamma) * u, gm1},
      {u * (0.5 * gm1 * u * u - H), H - gm1 * u * u, a.gamma * u}};
  double Ub[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double acc = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) acc += (wbp[c] + wbm[c]) * J[c][d];
    Ub[d] = 0.5 * acc + 0.5 * alpha * (wbp[d] - wbm[d]);
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int64_t gi = c * n + j;
    if (a.stage_mode == 0) {
      a.out[gi] = Ub[c];
    } else {
      const double dt = a.dt_arr[0];
      const double mu_j = MU[c][t + 3];
      const double v = mu_j + dt * Ub[c];
      const double ain = a.acc_in ? accv[c] : 0.0;
      a.out[gi] = a.p * v + a.q * ain;
      if (a.acc_out) a.acc_out[gi] = a.r * ain + a.s * mu_j;
    }
  }
}

static int launch_vjp(const VjpArgs& a, hipStream_t s) {
  const int64_t blocks = (a.n + VJP_TC - 1) / VJP_TC;
  if (blocks > 0x7fffffff) return set_error(WZN_ERR_SIZE, "grid too large (vjp)");
  hipLaunchKernelGGL(vjp_kernel, dim3((unsigned)blocks), dim3(VJP_NT), 0, s, a);
  return check_launch("vjp_kernel");
}

static VjpArgs vjp_base(const wzn_params* p, int64_t n, double dx) {
  VjpArgs a{};
  a.n = n;
  a.dx = dx;
  a.bc = p->bc_x;
  a.gamma = p->gamma;
  a.eps = p->eps;
  a.A = p->A;
  return a;
}

int rhs_1d_vjp(const wzn_params* p, const double* u, const double* mu, double* out, int64_t n,
               double dx, Workspace* ws, hipStream_t s) {
  VjpArgs a = vjp_base(p, n, dx);
  a.U = u;
  a.mu = mu;
  a.out = out;
  if (p->lf_alpha_x >= 0.0) {
    a.alpha_const = p->lf_alpha_x;
  } else {
    int st = launch_zero_words(ws->speed, 1, s);
    if (st) return st;
    st = launch_speed_max<double>(u, n, 3, p->gamma, ws->speed, nullptr, s);
    if (st) return st;
    a.alpha_arr = (const double*)ws->speed;  // the max, frozen
  }
  return launch_vjp(a, s);
}

int rk3_step_1d_vjp(const wzn_params* p, const double* stages, const double* lam_next,
                    double* lam_prev, double* scratch, int64_t n, double dx, const double* dt,
                    const double* alpha3, Workspace* ws, hipStream_t s) {
  (void)ws;
  const int64_t M = 3 * n;
  const double* U0 = stages;
  const double* U1 = stages + M;
  const double* U2 = stages + 2 * M;
  double* lam2 = scratch;
  double* lam1 = scratch + M;
  double* acc = scratch + 2 * M;
  // stage 3: lam2 = 2/3 (lam3 + dt J2^T lam3); acc = 1/3 lam3
  VjpArgs a = vjp_base(p, n, dx);
  a.stage_mode = 1;
  a.dt_arr = dt;
  a.U = U2;
  a.mu = lam_next;
  a.alpha_arr = alpha3 + 2;
  a.out = lam2;
  a.acc_in = nullptr;
  a.acc_out = acc;
  a.p = 2.0 / 3.0; a.q = 0.0; a.r = 0.0; a.s = 1.0 / 3.0;
  int st = launch_vjp(a, s);
  if (st) return st;
  // stage 2: lam1 = 1/4 (lam2 + dt J1^T lam2); acc += 3/4 lam2
  a.U = U1;
  a.mu = lam2;
  a.alpha_arr = alpha3 + 1;
  a.out = lam1;
  a.acc_in = acc;
  a.acc_out = acc;
  a.p = 0.25; a.q = 0.0; a.r = 1.0; a.s = 0.75;
  st = launch_vjp(a, s);
  if (st) return st;
  // stage 1: lam0 = acc + lam1 + dt J0^T lam1
  a.U = U0;
  a.mu = lam1;
  a.alpha_arr = alpha3;
  a.out = lam_prev;
  a.acc_in = acc;
  a.acc_out = nullptr;
  a.p = 1.0; a.q = 1.0; a.r = 0.0; a.s = 0.0;
  return launch_vjp(a, s);
}

// Three stage launches of one TVD-RK3 step with a frozen schedule, reading U^n from `uin`
// and writing U1, U2 and (unless uout is null) U^{n+1} to separate arrays.
static int frozen_step(const wzn_params* p, const double* uin, double* U1, double* U2,
                       double* uout, int64_t n, double dx, const double* dt,
                       const double* alpha3, hipStream_t s) {
  const double ra[3] = {0.0, 3.0 / 4.0, 1.0 / 3.0};
  const double rb[3] = {1.0, 1.0 / 4.0, 2.0 / 3.0};
  for (int k = 0; k < 3; ++k) {
    if (k == 2 && !uout) break;
    RowArgs<double> a{};
    a.n = n;
    a.plane = n;
    a.dx = dx;
    a.bc = p->bc_x;
    a.gamma = p->gamma;
    a.eps_s = 16.0 * p->eps;
    a.A = p->A;
    a.mode = MODE_STAGE;
    a.uin = k == 0 ? uin : (k == 1 ? U1 : U2);
    a.out = k == 0 ? U1 : (k == 1 ? U2 : uout);
    a.un = k == 0 ? nullptr : uin;
    a.rk_a = ra[k];
    a.rk_b = rb[k];
    a.alpha_arr = alpha3 + k;
    a.dt_arr = dt;
    int st = launch_rows(a, SYS_EULER1, 1, tuning_1d(3, n), s);
    if (st) return st;
  }
  return WZN_OK;
}

int rk3_adjoint_1d(const wzn_params* p, const double* ckpts, int32_t nsteps, int32_t ckpt_every,
                   const double* dts, const double* alphas, double* lam, double* work,
                   int64_t n, double dx, Workspace* ws, hipStream_t s) {
  const int64_t M = 3 * n;
  double* seg = work;                                  // [ckpt_every][3][M]
  double* scratch = work + (int64_t)ckpt_every * 3 * M;  // [3][M]
  double* lam_b = scratch + 3 * M;                     // [M]
  const int32_t nseg = (nsteps + ckpt_every - 1) / ckpt_every;
  double* cur = lam;
  double* other = lam_b;
  for (int32_t sg = nseg - 1; sg >= 0; --sg) {
    const int32_t t0 = sg * ckpt_every;
    const int32_t steps = nsteps - t0 < ckpt_every ? nsteps - t0 : ckpt_every;
    // recompute the stage states of the segment from its checkpoint
    for (int32_t k = 0; k < steps; ++k) {
      const double* uin = k == 0 ? ckpts + (int64_t)sg * M : seg + (int64_t)k * 3 * M;
      double* st_k = seg + (int64_t)k * 3 * M;
      double* uout = k + 1 < steps ? seg + (int64_t)(k + 1) * 3 * M : nullptr;
      if (k == 0) {
        if (hipMemcpyAsync(st_k, uin, sizeof(double) * M, hipMemcpyDeviceToDevice, s) !=
            hipSuccess)
          return set_error(WZN_ERR_HIP, "hipMemcpyAsync (checkpoint) failed");
      }
      int st = frozen_step(p, st_k, st_k + M, st_k + 2 * M, uout, n, dx, dts + t0 + k,
                           alphas + 3 * (int64_t)(t0 + k), s);
      if (st) return st;
    }
    // adjoint of the segment's steps, last to first
    for (int32_t k = steps - 1; k >= 0; --k) {
      int st = rk3_step_1d_vjp(p, seg + (int64_t)k * 3 * M, cur, other, scratch, n, dx,
                               dts + t0 + k, alphas + 3 * (int64_t)(t0 + k), ws, s);
      if (st) return st;
      double* tmp = cur;
      cur = other;
      other = tmp;
    }
  }
  if (cur != lam) {
    if (hipMemcpyAsync(lam, cur, sizeof(double) * M, hipMemcpyDeviceToDevice, s) != hipSuccess)
      return set_error(WZN_ERR_HIP, "hipMemcpyAsync (adjoint result) failed");
  }
  return WZN_OK;
}

}  // namespace wzn
