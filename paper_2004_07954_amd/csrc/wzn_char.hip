// 1D Euler with the WENO-ZN reconstruction carried out in local characteristic fields
// (Sec. 4.3): right-hand side and fused TVD-RK3 stages.
//
// For the interface x_{i+1/2} between cells i and i+1:
//   - the eigen-system of the flux Jacobian at the Roe average of U_i and U_{i+1}
//     (u and H = (E + p)/rho weighted by sqrt(rho), c^2 = (gamma - 1)(H - u^2/2)):
//     right eigenvectors (1, u - c, H - u c), (1, u, u^2/2), (1, u + c, H + u c) as the
//     columns of R, and Lc = R^{-1} in closed form with b1 = (gamma - 1)/c^2, b2 = b1 u^2/2;
//   - the six cells i-2 .. i+3 projected with that one Lc, and split field by field with
//     w^{+-}_k = Lc_k F +- alpha_k Lc_k U (= twice the split flux), alpha_k the global
//     max |lambda_k| of the RHS input, lambda = (u - c, u, u + c);
//   - ghat_k = WZN(w^+_k at cells i-2..i+2) + WZN(w^-_k at cells i+3..i-1) (mirrored), and the
//     interface flux R ghat / 2.
//
// Work mapping: one workgroup of NT threads owns NT consecutive interfaces (NT - 1 output
// cells; neighbouring tiles overlap by one interface).  Every cell of the tile and its halo
// is loaded once and its U, F, sqrt(rho), u and H are staged in LDS (structure of arrays, so
// lane t reading cell t + j touches consecutive words); each thread then builds the Roe
// eigen-system of its interface, projects the six stencil cells field by field, runs the six
// reconstructions, and writes R ghat to LDS, from which every output cell takes its two
// faces.  Nothing here is shared between interfaces: Lc differs from one to the next.
// Stage mode fuses the TVD-RK3 combination (the stage input U comes from LDS) and, on request,
// the per-field maxima |u - c|, |u|, |u + c| of the output (the next stage's alphas; their
// max(|u - c|, |u + c|) is the |u| + c of the CFL time step, bit for bit).
#include <hip/hip_runtime.h>

#include "wzn_device.hpp"
#include "wzn_host.hpp"
#include "wzn_rows.hpp"
#include "wzn_tile.hpp"

namespace wzn {

struct CharArgs {
  const double* uin;   // stage input [3][n]
  const double* un;    // U^n for the stage combination, or null when a_s == 0
  double* out;         // L (MODE_RHS) or U^(s+1) (MODE_STAGE), [3][n]
  int n;
  int bc;
  int mode;
  double dx, half_inv_dx, rk_a, rk_b, gamma, eps_s, Aq;
  // per-field alphas of this evaluation: 3 slots (reduced) / array of 3 (frozen) / constant
  const unsigned long long* alpha_slot;
  const double* alpha_arr;
  double alpha_const;
  // dt: array / cfl dx / max(slot[0], slot[2]) / the dt slot
  const double* dt_arr;
  const unsigned long long* dt_speed_slot;
  const double* dt_slot_read;
  double cfl;
  double* dt_slot_write;
  double* dt_rec;
  double* alpha_rec;                // [3] or null
  unsigned long long* speed_next;   // [3]: atomic max of |u - c|, |u|, |u + c| of the output
  unsigned long long* slot_zero;    // [3] zeroed by workgroup 0, or null
};

// staged per-cell planes
enum { CP_U0 = 0, CP_F0 = 3, CP_S = 6, CP_V = 7, CP_H = 8, CP_N = 9 };

// |u - c|, |u|, |u + c| of a 1D Euler state, with c as in wave_speed_1d (same operations).
__device__ __forceinline__ void char_speeds(double rho, double m, double E, double gamma,
                                            double& s0, double& s1, double& s2) {
#pragma clang fp contract(off)
  const double r = rcp_nr(rho);
  const double u = m * r;
  const double p = (gamma - 1.0) * (E - (0.5 * m) * u);
  const double c = sqrt_gs((gamma * p) * r);
  s0 = __builtin_fabs(u - c);
  s1 = __builtin_fabs(u);
  s2 = __builtin_fabs(u + c);
}

// Launch shape: threads (= interfaces) per workgroup; FIELD_OUTER projects and reconstructs one
// field at a time, re-reading the stencil from LDS for each (78 VGPRs, six waves per SIMD),
// instead of projecting all three fields first (124 VGPRs, four waves); WAVES_PER_EU is the
// occupancy the register allocation must allow.  Measured on MI355X at 2^20 cells: 256 threads
// field-outer 35.1 us per stage, all fields first 37.1 us, 128 threads 38.0-38.3 us, 64
// threads 42.2 us (the same bits in every case).
constexpr int CHAR_NT = 256;
constexpr bool CHAR_FIELD_OUTER = true;
constexpr int CHAR_WAVES_PER_EU = 1;

template <int NT, bool FIELD_OUTER>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(CHAR_WAVES_PER_EU)))
void char_kernel(CharArgs a) {
  constexpr int NC = NT + 5;  // cells c0 - 3 .. c0 + NT + 1
  __shared__ double S[CP_N][NC];
  __shared__ double FH[3][NT];
  __shared__ double red[3][NT / 64];
  const int tid = threadIdx.x;
  const int64_t pl = a.n;

  double al[3];
#pragma unroll
  for (int f = 0; f < 3; ++f)
    al[f] = a.alpha_slot ? slot_value(a.alpha_slot + f)
                         : (a.alpha_arr ? a.alpha_arr[f] : a.alpha_const);
  double dt = 0.0;
  if (a.mode == MODE_STAGE) {
    if (a.dt_arr) dt = a.dt_arr[0];
    else if (a.dt_speed_slot)
      dt = a.cfl * a.dx / fmax(slot_value(a.dt_speed_slot), slot_value(a.dt_speed_slot + 2));
    else dt = a.dt_slot_read[0];
  }
  if (blockIdx.x == 0 && tid == 0) {
    if (a.dt_slot_write) a.dt_slot_write[0] = dt;
    if (a.dt_rec) a.dt_rec[0] = dt;
    if (a.alpha_rec)
      for (int f = 0; f < 3; ++f) a.alpha_rec[f] = al[f];
    if (a.slot_zero)
      for (int f = 0; f < 3; ++f) a.slot_zero[f] = 0ull;
  }

  // ---- stage the tile's cells and halo (boundary conditions as an index map)
  const int c0 = blockIdx.x * (NT - 1);
  const double gm1 = a.gamma - 1.0;
  for (int l = tid; l < NC; l += NT) {
    const int ci = bc_cell(c0 - 3 + l, a.n, a.bc);
    const double rho = a.uin[ci], m = a.uin[pl + ci], E = a.uin[2 * pl + ci];
    double u, p;
    euler1_prim<double>(rho, m, E, gm1, u, p);
    S[CP_U0][l] = rho;
    S[CP_U0 + 1][l] = m;
    S[CP_U0 + 2][l] = E;
#pragma unroll
    for (int v = 0; v < 3; ++v) S[CP_F0 + v][l] = euler1_flux_comp<double>(v, m, E, u, p);
    S[CP_S][l] = sqrt_gs(rho);
    S[CP_V][l] = u;
    S[CP_H][l] = (E + p) * rcp_nr(rho);
  }
  __syncthreads();

  // ---- interface t: x_{c0 + t - 1/2}, stencil cells t .. t+5 of the staged tile
  {
    const int t = tid;
    const double sL = S[CP_S][t + 2], sR = S[CP_S][t + 3];
    const double wl = sL * rcp_nr(sL + sR);
    const double uh = fma_t(wl, S[CP_V][t + 2] - S[CP_V][t + 3], S[CP_V][t + 3]);
    const double Hh = fma_t(wl, S[CP_H][t + 2] - S[CP_H][t + 3], S[CP_H][t + 3]);
    const double c = sqrt_gs(gm1 * fma_t(-0.5 * uh, uh, Hh));
    const double ic = rcp_nr(c);
    const double b1 = (gm1 * ic) * ic;
    const double b1u = b1 * uh;
    const double b2 = (0.5 * b1u) * uh;
    const double uic = uh * ic;
    const double Lc[3][3] = {{0.5 * (b2 + uic), -0.5 * (b1u + ic), 0.5 * b1},
                             {1.0 - b2, b1u, -b1},
                             {0.5 * (b2 - uic), -0.5 * (b1u - ic), 0.5 * b1}};
    // w^+ over cells 0..4, w^- over cells 5..1 (mirrored window)
    double gh[3];
    if constexpr (!FIELD_OUTER) {
      double wp[3][5], wm[3][5];
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        const double U0 = S[CP_U0][t + j], U1 = S[CP_U0 + 1][t + j], U2 = S[CP_U0 + 2][t + j];
        const double F0 = S[CP_F0][t + j], F1 = S[CP_F0 + 1][t + j], F2 = S[CP_F0 + 2][t + j];
#pragma unroll
        for (int f = 0; f < 3; ++f) {
          const double V = fma_t(Lc[f][2], U2, fma_t(Lc[f][1], U1, Lc[f][0] * U0));
          const double G = fma_t(Lc[f][2], F2, fma_t(Lc[f][1], F1, Lc[f][0] * F0));
          if (j < 5) wp[f][j] = fma_t(al[f], V, G);
          if (j > 0) wm[f][5 - j] = fma_t(-al[f], V, G);
        }
      }
#pragma unroll
      for (int f = 0; f < 3; ++f) {
        double hp, hm;
        wzn_window<1>(wp[f], &hp, a.eps_s, a.Aq);
        wzn_window<1>(wm[f], &hm, a.eps_s, a.Aq);
        gh[f] = hp + hm;
      }
    } else {
#pragma unroll
      for (int f = 0; f < 3; ++f) {
        // a compiler memory barrier: the stencil is read again from LDS for every field
        // rather than held in registers across the three
        if (f > 0) asm volatile("" ::: "memory");
        double wp[5], wm[5];
#pragma unroll
        for (int j = 0; j < 6; ++j) {
          const double V = fma_t(Lc[f][2], S[CP_U0 + 2][t + j],
                                 fma_t(Lc[f][1], S[CP_U0 + 1][t + j], Lc[f][0] * S[CP_U0][t + j]));
          const double G = fma_t(Lc[f][2], S[CP_F0 + 2][t + j],
                                 fma_t(Lc[f][1], S[CP_F0 + 1][t + j], Lc[f][0] * S[CP_F0][t + j]));
          if (j < 5) wp[j] = fma_t(al[f], V, G);
          if (j > 0) wm[5 - j] = fma_t(-al[f], V, G);
        }
        double hp, hm;
        wzn_window<1>(wp, &hp, a.eps_s, a.Aq);
        wzn_window<1>(wm, &hm, a.eps_s, a.Aq);
        gh[f] = hp + hm;
      }
    }
    const double uc = uh * c;
    FH[0][t] = gh[0] + gh[1] + gh[2];
    FH[1][t] = fma_t(uh - c, gh[0], fma_t(uh, gh[1], (uh + c) * gh[2]));
    FH[2][t] = fma_t(Hh - uc, gh[0], fma_t((0.5 * uh) * uh, gh[1], (Hh + uc) * gh[2]));
  }
  __syncthreads();

  // ---- output cell c0 + t: faces t (left) and t + 1 (right); FH holds twice the flux
  double sp[3] = {0.0, 0.0, 0.0};
  const int i = c0 + tid;
  if (tid < NT - 1 && i < a.n) {
    const double sc = a.half_inv_dx;
    double o[3];
#pragma unroll
    for (int v = 0; v < 3; ++v) {
      const double L = (FH[v][tid] - FH[v][tid + 1]) * sc;
      if (a.mode == MODE_RHS) {
        o[v] = L;
      } else {
        double base = a.rk_b * S[CP_U0 + v][tid + 3];
        if (a.un) base = fma_t(a.rk_a, a.un[v * pl + i], base);
        o[v] = fma_t(a.rk_b * dt, L, base);
      }
      a.out[v * pl + i] = o[v];
    }
    if (a.speed_next) char_speeds(o[0], o[1], o[2], a.gamma, sp[0], sp[1], sp[2]);
  }
  if (a.speed_next) {
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      const double m = wave_max(sp[f]);
      if ((tid & 63) == 0) red[f][tid >> 6] = m;
    }
    __syncthreads();
    if (tid < 3) {
      double m = 0.0;
#pragma unroll
      for (int w = 0; w < NT / 64; ++w) m = fmax(m, red[tid][w]);
      atomic_max_pos(a.speed_next + tid, m);
    }
  }
}

// per-field maxima |u - c|, |u|, |u + c| over the cells of u into slot[0..2] (zero beforehand)
__global__ __launch_bounds__(256) void char_speed_kernel(const double* __restrict__ u, int n,
                                                         double gamma, unsigned long long* slot) {
  double s[3] = {0.0, 0.0, 0.0};
  const int64_t pl = n;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256) {
    double a0, a1, a2;
    char_speeds(u[i], u[pl + i], u[2 * pl + i], gamma, a0, a1, a2);
    s[0] = fmax(s[0], a0);
    s[1] = fmax(s[1], a1);
    s[2] = fmax(s[2], a2);
  }
  __shared__ double red[3][4];
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    const double m = wave_max(s[f]);
    if ((threadIdx.x & 63) == 0) red[f][threadIdx.x >> 6] = m;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    const int f = threadIdx.x;
    atomic_max_pos(slot + f, fmax(fmax(red[f][0], red[f][1]), fmax(red[f][2], red[f][3])));
  }
}

// ------------------------------------------------------------------ host side
static int launch_char(const CharArgs& a, hipStream_t s) {
  const int64_t blocks = ((int64_t)a.n + CHAR_NT - 2) / (CHAR_NT - 1);
  hipLaunchKernelGGL((char_kernel<CHAR_NT, CHAR_FIELD_OUTER>), dim3((unsigned)blocks),
                     dim3(CHAR_NT), 0, s, a);
  return check_launch("char_kernel");
}

static int launch_char_speed(const double* u, int n, double gamma, unsigned long long* slot,
                             hipStream_t s) {
  int64_t blocks = ((int64_t)n + 255) / 256;
  if (blocks > 2048) blocks = 2048;
  hipLaunchKernelGGL(char_speed_kernel, dim3((unsigned)blocks), dim3(256), 0, s, u, n, gamma,
                     slot);
  return check_launch("char_speed_kernel");
}

static CharArgs char_base(const wzn_params* p, int64_t n, double dx) {
  CharArgs a{};
  a.n = (int)n;
  a.bc = p->bc_x;
  a.dx = dx;
  a.half_inv_dx = 0.5 / dx;
  a.gamma = p->gamma;
  a.eps_s = 16.0 * p->eps;
  a.Aq = 0.25 * p->A;
  return a;
}

int rhs_1d_char(const wzn_params* p, const double* u, double* dudt, int64_t n, double dx,
                const double* alpha3, Workspace* ws, hipStream_t s) {
  CharArgs a = char_base(p, n, dx);
  a.uin = u;
  a.out = dudt;
  a.mode = MODE_RHS;
  if (alpha3) {
    a.alpha_arr = alpha3;
  } else if (p->lf_alpha_x >= 0.0) {
    a.alpha_const = p->lf_alpha_x;
  } else {
    int st = launch_zero_words(ws->char_speed, 3, s);
    if (st) return st;
    st = launch_char_speed(u, (int)n, p->gamma, ws->char_speed, s);
    if (st) return st;
    a.alpha_slot = ws->char_speed;
  }
  return launch_char(a, s);
}

// Same slot protocol as the component-wise run, with a ring of three triples: kernel s reads
// the per-field alphas of its input from triple s % 3 (and, at the first stage of a step, the
// dt speed max(slot[0], slot[2])), maxes those of its output into triple (s + 1) % 3, and
// clears triple (s + 2) % 3.
int rk3_run_1d_char(const wzn_params* p, double* u, double* stage, int64_t n, double dx,
                    double cfl, int32_t nsteps, const double* dt_in, const double* alpha_in,
                    double* dt_out, double* alpha_out, Workspace* ws, hipStream_t s) {
  static const double RA[3] = {0.0, 3.0 / 4.0, 1.0 / 3.0};
  static const double RB[3] = {1.0, 1.0 / 4.0, 2.0 / 3.0};
  const int64_t M = 3 * n;
  double* U1 = stage;
  double* U2 = stage + M;
  const bool reduce_alpha = alpha_in == nullptr && p->lf_alpha_x < 0.0;
  const bool cfl_dt = dt_in == nullptr;
  const bool need_speed = reduce_alpha || cfl_dt;
  unsigned long long* ring = ws->char_speed;
  int st = WZN_OK;
  if (need_speed && nsteps > 0) {
    st = launch_zero_words(ring, 9, s);
    if (st) return st;
    st = launch_char_speed(u, (int)n, p->gamma, ring, s);
    if (st) return st;
  }
  int64_t sidx = 0;
  for (int32_t step = 0; step < nsteps; ++step) {
    for (int k = 0; k < 3; ++k, ++sidx) {
      CharArgs a = char_base(p, n, dx);
      a.mode = MODE_STAGE;
      a.uin = k == 0 ? u : (k == 1 ? U1 : U2);
      a.out = k == 0 ? U1 : (k == 1 ? U2 : u);
      a.un = k == 0 ? nullptr : u;
      a.rk_a = RA[k];
      a.rk_b = RB[k];
      unsigned long long* cur = ring + 3 * (sidx % 3);
      if (alpha_in) a.alpha_arr = alpha_in + 9 * (int64_t)step + 3 * k;
      else if (reduce_alpha) a.alpha_slot = cur;
      else a.alpha_const = p->lf_alpha_x;
      if (dt_in) {
        a.dt_arr = dt_in + step;
      } else if (k == 0) {
        a.dt_speed_slot = cur;
        a.cfl = cfl;
        a.dt_slot_write = ws->dt;
      } else {
        a.dt_slot_read = ws->dt;
      }
      if (dt_out && k == 0) a.dt_rec = dt_out + step;
      if (alpha_out) a.alpha_rec = alpha_out + 9 * (int64_t)step + 3 * k;
      if (need_speed) {
        // with frozen alphas only U^{n+1} (k == 2) feeds a triple, for the next step's dt
        if (reduce_alpha || k == 2) a.speed_next = ring + 3 * ((sidx + 1) % 3);
        a.slot_zero = ring + 3 * ((sidx + 2) % 3);
      }
      st = launch_char(a, s);
      if (st) return st;
    }
  }
  return WZN_OK;
}

}  // namespace wzn
