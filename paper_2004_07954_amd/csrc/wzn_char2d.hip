// 2D Euler with each sweep's WENO-ZN reconstruction in local characteristic fields: the
// procedure of Sec. 4.3 applied along x and along y of the dimension-by-dimension scheme
// (eq:2d), with the time step of Sec. 4.4.
//
// At an x interface the flux Jacobian dF/dU is taken at the Roe average of the two
// neighbouring states (u, v, H = (E + p)/rho weighted by sqrt(rho); c^2 = (gamma - 1)(H -
// (u^2 + v^2)/2)).  Its eigenvalues are u - c, u, u, u + c; the right eigenvectors
// (1, u - c, v, H - u c), (1, u, v, (u^2 + v^2)/2), (0, 0, 1, v), (1, u + c, v, H + u c) are the
// columns of R, and Lc = R^{-1} in closed form with b1 = (gamma - 1)/c^2, b2 = b1 (u^2 + v^2)/2.
// The six stencil cells are projected with that one Lc and split field by field,
// w^{+-}_k = Lc_k F +- alpha_k Lc_k U (twice the split flux), alpha_k the global max of |u - c|,
// |u|, |u|, |u + c| over the cells of the RHS input; ghat_k = WZN(w^+_k) + WZN(w^-_k mirrored)
// and the interface flux is R ghat / 2.
//
// The y sweep is the same procedure on the state with the two momenta exchanged: the y
// Jacobian of U is the x Jacobian of the exchanged state, and the exchange flips only the sign
// of the shear eigenvector, which cancels in R ghat because the reconstruction is an odd
// function of its data.  A column kernel evaluates it in place, walking the columns of U (no
// transposed copy).  One right-hand side is: the column kernel -> Ly; then the x sweep of U,
// whose epilogue adds Ly and writes L, or the TVD-RK3 stage combination (U from LDS) with the
// per-field maxima of the output for the next stage's alphas and the next step's dt.
#include <hip/hip_runtime.h>

#include "wzn_device.hpp"
#include "wzn_host.hpp"
#include "wzn_rows.hpp"
#include "wzn_tile.hpp"

namespace wzn {

struct Char2Args {
  const double* uin;   // [4][rows][n]
  double* out;         // [4][rows][n]: this sweep's part of L
  int n;               // cells per row
  int64_t rows;
  int64_t tiles;       // workgroups per row
  int64_t plane;       // rows * n
  int bc;
  double half_inv_h, gamma, eps_s, Aq;
  // per-field alphas: 3 slots (max |un - c|, |un|, |un + c|) / array of 4 / constant
  const unsigned long long* alpha_slot;
  const double* alpha_arr;
  double alpha_const;
  unsigned long long* slot_zero;  // words cleared by workgroup 0, or null
  int zero_count;
  // FUSE (the x sweep): the epilogue adds ly [4][rows][n] (the y part of L) and writes L
  // (MODE_RHS) or the TVD-RK3 stage output, with the per-field maxima of the output
  const double* ly;
  const double* un;    // U^n or null
  int mode;
  double rk_a, rk_b;
  const double* dt_arr;                   // dt: array /
  const unsigned long long* dt_speed_slot;  // cfl dtx dty / (dtx + dty) from six slots /
  const double* dt_slot_read;             // the dt slot
  double cfl, dx, dy;
  double* dt_slot_write;
  double* dt_rec;
  unsigned long long* speed_next;  // [6] maxima of the output, or null
};

// staged per-cell planes
enum { C2_U0 = 0, C2_F0 = 4, C2_S = 8, C2_VU = 9, C2_VV = 10, C2_H = 11, C2_N = 12 };
constexpr int C2_NT = 256;
// column kernel (the y sweep): CY_TX columns x CY_TY interfaces per workgroup
constexpr int CY_TX = 16, CY_TY = 16;

__device__ __forceinline__ void char2_speeds(double rho, double mx, double my, double E,
                                             double gamma, double (&s)[6]);
__device__ __forceinline__ void block_max6(double (&s)[6], unsigned long long* slot);

// The sweep's alphas for the four fields (Sec. 4.3: one per field, |un - c|, |un|, |un|,
// |un + c|) from three slots, a device array of four or one constant.
__device__ __forceinline__ void char2_alphas(const Char2Args& a, double (&al)[4]) {
  if (a.alpha_slot) {
    al[0] = slot_value(a.alpha_slot);
    al[1] = al[2] = slot_value(a.alpha_slot + 1);
    al[3] = slot_value(a.alpha_slot + 2);
  } else if (a.alpha_arr) {
#pragma unroll
    for (int f = 0; f < 4; ++f) al[f] = a.alpha_arr[f];
  } else {
#pragma unroll
    for (int f = 0; f < 4; ++f) al[f] = a.alpha_const;
  }
}

// Stage one cell of a sweep at LDS position l (planes PS elements apart): U, the flux along
// the sweep F = (mn, mn un + p, mn ut, un (E + p)), sqrt(rho), un, ut and H = (E + p) / rho,
// where mn / mt are the normal / tangential momenta (mx / my in the x sweep, my / mx in the
// y sweep, which is how the y sweep becomes the x procedure of the exchanged state).
template <int PS>
__device__ __forceinline__ void char2_stage(double* S, int l, double rho, double mn, double mt,
                                            double E, double gm1) {
  const double r = rcp_nr(rho);
  const double u = mn * r, v = mt * r;
  const double p = gm1 * fma_t(-(0.5 * mt), v, fma_t(-(0.5 * mn), u, E));
  S[C2_U0 * PS + l] = rho;
  S[(C2_U0 + 1) * PS + l] = mn;
  S[(C2_U0 + 2) * PS + l] = mt;
  S[(C2_U0 + 3) * PS + l] = E;
  S[C2_F0 * PS + l] = mn;
  S[(C2_F0 + 1) * PS + l] = fma_t(mn, u, p);
  S[(C2_F0 + 2) * PS + l] = mn * v;
  S[(C2_F0 + 3) * PS + l] = u * (E + p);
  S[C2_S * PS + l] = sqrt_gs(rho);
  S[C2_VU * PS + l] = u;
  S[C2_VV * PS + l] = v;
  S[C2_H * PS + l] = (E + p) * r;
}

// Twice the interface flux R ghat (normal-first component order) of the interface between
// stencil cells 2 and 3, the six cells at LDS positions t, t + ES, ..., t + 5 ES.
template <int PS, int ES>
__device__ __forceinline__ void char2_face(const double* S, int t, const double (&al)[4],
                                           double gm1, double eps_s, double Aq,
                                           double (&fh)[4]) {
#define SV(pl, j) S[(pl) * PS + t + (j) * ES]
  const double sL = SV(C2_S, 2), sR = SV(C2_S, 3);
  const double wl = sL * rcp_nr(sL + sR);
  const double uh = fma_t(wl, SV(C2_VU, 2) - SV(C2_VU, 3), SV(C2_VU, 3));
  const double vh = fma_t(wl, SV(C2_VV, 2) - SV(C2_VV, 3), SV(C2_VV, 3));
  const double Hh = fma_t(wl, SV(C2_H, 2) - SV(C2_H, 3), SV(C2_H, 3));
  const double q2 = fma_t(uh, uh, vh * vh);
  const double c = sqrt_gs(gm1 * fma_t(-0.5, q2, Hh));
  const double ic = rcp_nr(c);
  const double b1 = (gm1 * ic) * ic;
  const double b1u = b1 * uh, b1v = b1 * vh;
  const double b2 = (0.5 * b1) * q2;
  const double uic = uh * ic;
  // rows 0, 1, 3 of Lc (row 2, the shear field, is (-v, 0, 1, 0))
  const double Lc[4][4] = {{0.5 * (b2 + uic), -0.5 * (b1u + ic), -0.5 * b1v, 0.5 * b1},
                           {1.0 - b2, b1u, b1v, -b1},
                           {0.0, 0.0, 0.0, 0.0},
                           {0.5 * (b2 - uic), -0.5 * (b1u - ic), -0.5 * b1v, 0.5 * b1}};
  double gh[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    // a compiler memory barrier: the stencil is read again from LDS for every field
    if (f > 0) asm volatile("" ::: "memory");
    double wp[5], wm[5];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      double V, G;
      if (f == 2) {
        V = fma_t(-vh, SV(C2_U0, j), SV(C2_U0 + 2, j));
        G = fma_t(-vh, SV(C2_F0, j), SV(C2_F0 + 2, j));
      } else {
        V = fma_t(Lc[f][3], SV(C2_U0 + 3, j),
                  fma_t(Lc[f][2], SV(C2_U0 + 2, j),
                        fma_t(Lc[f][1], SV(C2_U0 + 1, j), Lc[f][0] * SV(C2_U0, j))));
        G = fma_t(Lc[f][3], SV(C2_F0 + 3, j),
                  fma_t(Lc[f][2], SV(C2_F0 + 2, j),
                        fma_t(Lc[f][1], SV(C2_F0 + 1, j), Lc[f][0] * SV(C2_F0, j))));
      }
      if (j < 5) wp[j] = fma_t(al[f], V, G);
      if (j > 0) wm[5 - j] = fma_t(-al[f], V, G);
    }
    double hp, hm;
    wzn_window<1>(wp, &hp, eps_s, Aq);
    wzn_window<1>(wm, &hm, eps_s, Aq);
    gh[f] = hp + hm;
    // materialise here: otherwise every field's arithmetic is sunk below the last field's
    // loads and all four fields' stencils are live at once (twice the registers)
    asm volatile("" : "+v"(gh[f]));
  }
#undef SV
  const double uc = uh * c;
  fh[0] = (gh[0] + gh[1]) + gh[3];
  fh[1] = fma_t(uh - c, gh[0], fma_t(uh, gh[1], (uh + c) * gh[3]));
  fh[2] = fma_t(vh, gh[0] + gh[1] + gh[3], gh[2]);
  fh[3] = fma_t(Hh - uc, gh[0], fma_t(0.5 * q2, gh[1], fma_t(vh, gh[2], (Hh + uc) * gh[3])));
}

// The x sweep.  One workgroup: NT interfaces of one row (NT - 1 output cells; neighbouring
// tiles overlap by one interface).  Every cell of the tile and its halo is loaded once and its
// U, F, sqrt(rho), u, v and H are staged in LDS; each thread builds the Roe eigen-system of its
// interface and reconstructs the four fields one after another, re-reading the stencil from
// LDS for each.  FUSE: the epilogue adds the y part and forms L or the stage output.  (The
// same face as char2_face, written out: with the helper the compiler keeps ten more registers
// live here and the fused kernel drops from four waves per SIMD to three.)
template <int NT, bool FUSE>
__global__ __launch_bounds__(NT) void char2_kernel(Char2Args a) {
  constexpr int NC = NT + 5;  // cells c0 - 3 .. c0 + NT + 1
  __shared__ double S[C2_N][NC];
  __shared__ double FH[4][NT];
  const int tid = threadIdx.x;
  const int64_t row = (int64_t)blockIdx.x / a.tiles;
  const int tile = (int)((int64_t)blockIdx.x - row * a.tiles);
  const double* uin = a.uin + row * a.n;

  double al[4];
  if (a.alpha_slot) {
    al[0] = slot_value(a.alpha_slot);
    al[1] = al[2] = slot_value(a.alpha_slot + 1);
    al[3] = slot_value(a.alpha_slot + 2);
  } else if (a.alpha_arr) {
#pragma unroll
    for (int f = 0; f < 4; ++f) al[f] = a.alpha_arr[f];
  } else {
#pragma unroll
    for (int f = 0; f < 4; ++f) al[f] = a.alpha_const;
  }
  if (blockIdx.x == 0 && a.slot_zero && tid < a.zero_count) a.slot_zero[tid] = 0ull;

  // ---- stage the tile's cells and halo (boundary conditions as an index map)
  const int c0 = tile * (NT - 1);
  const double gm1 = a.gamma - 1.0;
  for (int l = tid; l < NC; l += NT) {
    const int ci = bc_cell(c0 - 3 + l, a.n, a.bc);
    const double rho = uin[ci], mx = uin[a.plane + ci], my = uin[2 * a.plane + ci],
                 E = uin[3 * a.plane + ci];
    const double r = rcp_nr(rho);
    const double u = mx * r, v = my * r;
    const double p = gm1 * fma_t(-(0.5 * my), v, fma_t(-(0.5 * mx), u, E));
    S[C2_U0][l] = rho;
    S[C2_U0 + 1][l] = mx;
    S[C2_U0 + 2][l] = my;
    S[C2_U0 + 3][l] = E;
    S[C2_F0][l] = mx;
    S[C2_F0 + 1][l] = fma_t(mx, u, p);
    S[C2_F0 + 2][l] = mx * v;
    S[C2_F0 + 3][l] = u * (E + p);
    S[C2_S][l] = sqrt_gs(rho);
    S[C2_VU][l] = u;
    S[C2_VV][l] = v;
    S[C2_H][l] = (E + p) * r;
  }
  // (FUSE) the epilogue's loads of the y part and of U^n are issued now, so that they are in
  // flight during the reconstructions
  const int i = c0 + tid;
  const bool owns = tid < NT - 1 && i < a.n;
  const int64_t gi = row * a.n + (owns ? i : 0);
  double lyv[4] = {0.0, 0.0, 0.0, 0.0}, unv[4] = {0.0, 0.0, 0.0, 0.0};
  if constexpr (FUSE) {
    if (owns) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        lyv[v] = a.ly[v * a.plane + gi];
        if (a.un) unv[v] = a.un[v * a.plane + gi];
      }
    }
  }
  __syncthreads();

  // ---- interface t: x_{c0 + t - 1/2}, stencil cells t .. t+5 of the staged tile
  {
    const int t = tid;
    const double sL = S[C2_S][t + 2], sR = S[C2_S][t + 3];
    const double wl = sL * rcp_nr(sL + sR);
    const double uh = fma_t(wl, S[C2_VU][t + 2] - S[C2_VU][t + 3], S[C2_VU][t + 3]);
    const double vh = fma_t(wl, S[C2_VV][t + 2] - S[C2_VV][t + 3], S[C2_VV][t + 3]);
    const double Hh = fma_t(wl, S[C2_H][t + 2] - S[C2_H][t + 3], S[C2_H][t + 3]);
    const double q2 = fma_t(uh, uh, vh * vh);
    const double c = sqrt_gs(gm1 * fma_t(-0.5, q2, Hh));
    const double ic = rcp_nr(c);
    const double b1 = (gm1 * ic) * ic;
    const double b1u = b1 * uh, b1v = b1 * vh;
    const double b2 = (0.5 * b1) * q2;
    const double uic = uh * ic;
    // rows 0, 1, 3 of Lc (row 2, the shear field, is (-v, 0, 1, 0))
    const double Lc[4][4] = {{0.5 * (b2 + uic), -0.5 * (b1u + ic), -0.5 * b1v, 0.5 * b1},
                             {1.0 - b2, b1u, b1v, -b1},
                             {0.0, 0.0, 0.0, 0.0},
                             {0.5 * (b2 - uic), -0.5 * (b1u - ic), -0.5 * b1v, 0.5 * b1}};
    double gh[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      // a compiler memory barrier: the stencil is read again from LDS for every field
      if (f > 0) asm volatile("" ::: "memory");
      double wp[5], wm[5];
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        double V, G;
        if (f == 2) {
          V = fma_t(-vh, S[C2_U0][t + j], S[C2_U0 + 2][t + j]);
          G = fma_t(-vh, S[C2_F0][t + j], S[C2_F0 + 2][t + j]);
        } else {
          V = fma_t(Lc[f][3], S[C2_U0 + 3][t + j],
                    fma_t(Lc[f][2], S[C2_U0 + 2][t + j],
                          fma_t(Lc[f][1], S[C2_U0 + 1][t + j], Lc[f][0] * S[C2_U0][t + j])));
          G = fma_t(Lc[f][3], S[C2_F0 + 3][t + j],
                    fma_t(Lc[f][2], S[C2_F0 + 2][t + j],
                          fma_t(Lc[f][1], S[C2_F0 + 1][t + j], Lc[f][0] * S[C2_F0][t + j])));
        }
        if (j < 5) wp[j] = fma_t(al[f], V, G);
        if (j > 0) wm[5 - j] = fma_t(-al[f], V, G);
      }
      double hp, hm;
      wzn_window<1>(wp, &hp, a.eps_s, a.Aq);
      wzn_window<1>(wm, &hm, a.eps_s, a.Aq);
      gh[f] = hp + hm;
    }
    const double uc = uh * c;
    FH[0][t] = (gh[0] + gh[1]) + gh[3];
    FH[1][t] = fma_t(uh - c, gh[0], fma_t(uh, gh[1], (uh + c) * gh[3]));
    FH[2][t] = fma_t(vh, gh[0] + gh[1] + gh[3], gh[2]);
    FH[3][t] = fma_t(Hh - uc, gh[0],
                     fma_t(0.5 * q2, gh[1], fma_t(vh, gh[2], (Hh + uc) * gh[3])));
  }
  __syncthreads();

  // ---- output cell c0 + t: faces t (left) and t + 1 (right); FH holds twice the flux
  if constexpr (!FUSE) {
    (void)lyv;
    (void)unv;
    if (owns) {
      double* out = a.out + row * a.n + i;
#pragma unroll
      for (int v = 0; v < 4; ++v)
        out[v * a.plane] = (FH[v][tid] - FH[v][tid + 1]) * a.half_inv_h;
    }
  } else {
    double dt = 0.0;
    if (a.mode == MODE_STAGE) {
      if (a.dt_arr) {
        dt = a.dt_arr[0];
      } else if (a.dt_speed_slot) {
        // max(|u - c|, |u + c|) is |u| + c bit for bit, likewise for v
        const double sx = fmax(slot_value(a.dt_speed_slot), slot_value(a.dt_speed_slot + 2));
        const double sy =
            fmax(slot_value(a.dt_speed_slot + 3), slot_value(a.dt_speed_slot + 5));
        const double dtx = a.dx / sx, dty = a.dy / sy;
        dt = a.cfl * dtx * dty / (dtx + dty);
      } else {
        dt = a.dt_slot_read[0];
      }
    }
    if (blockIdx.x == 0 && tid == 0) {
      if (a.dt_slot_write) a.dt_slot_write[0] = dt;
      if (a.dt_rec) a.dt_rec[0] = dt;
    }
    double m[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (owns) {
      // (no contraction: the x part is rounded before the y part is added, as the y part
      // was, so that exchanging x and y gives the same bits)
#pragma clang fp contract(off)
      double o[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double lxv = (FH[v][tid] - FH[v][tid + 1]) * a.half_inv_h;
        const double L = lxv + lyv[v];
        if (a.mode == MODE_RHS) {
          o[v] = L;
        } else {
          double base = a.rk_b * S[C2_U0 + v][tid + 3];
          if (a.un) base = fma_t(a.rk_a, unv[v], base);
          o[v] = fma_t(a.rk_b * dt, L, base);
        }
        a.out[v * a.plane + gi] = o[v];
      }
      if (a.speed_next) char2_speeds(o[0], o[1], o[2], o[3], a.gamma, m);
    }
    // (the staged planes are no longer read: their LDS holds the reduction)
    if (a.speed_next) block_max_lds<NT, 6>(m, &S[0][0], a.speed_next);
  }
}

// The y sweep, walking the columns of the untransposed state u[4][ny][nx] (a.n = ny cells per
// column, a.rows = nx columns, a.tiles = tiles per column).  One workgroup: TX consecutive
// columns x TY interfaces of each (TY - 1 output cells; tiles overlap by one interface along
// y).  The tile's cells and its 3 + 2 halo rows are staged once, row segments of TX cells
// loaded together; thread (column x, interface t) evaluates the same face as the x sweep of
// the exchanged state (my as the normal momentum), and writes its part of L with the momenta
// back in place.
template <int TX, int TY>
__global__ __launch_bounds__(TX * TY) void char2_col_kernel(Char2Args a) {
  constexpr int NR = TY + 5;     // rows y0 - 3 .. y0 + TY + 1
  constexpr int PS = NR * TX;    // elements per staged plane
  __shared__ double S[C2_N * PS];
  __shared__ double FH[4][TY * TX];
  const int tid = threadIdx.x;
  const int64_t nx = a.rows;
  const int64_t cblk = (int64_t)blockIdx.x / a.tiles;
  const int tile = (int)((int64_t)blockIdx.x - cblk * a.tiles);
  const int64_t x0 = cblk * TX;

  double al[4];
  char2_alphas(a, al);
  if (blockIdx.x == 0 && a.slot_zero && tid < a.zero_count) a.slot_zero[tid] = 0ull;

  const int y0 = tile * (TY - 1);
  const double gm1 = a.gamma - 1.0;
  for (int l = tid; l < PS; l += TX * TY) {
    const int r = l / TX, cx = l - r * TX;
    const int64_t x = x0 + cx < nx ? x0 + cx : nx - 1;  // columns past the grid: any cell
    const int64_t ci = (int64_t)bc_cell(y0 - 3 + r, a.n, a.bc) * nx + x;
    char2_stage<PS>(S, l, a.uin[ci], a.uin[2 * a.plane + ci], a.uin[a.plane + ci],
                    a.uin[3 * a.plane + ci], gm1);
  }
  __syncthreads();

  const int cx = tid % TX, t = tid / TX;
  {
    double fh[4];
    char2_face<PS, TX>(S, t * TX + cx, al, gm1, a.eps_s, a.Aq, fh);
#pragma unroll
    for (int v = 0; v < 4; ++v) FH[v][tid] = fh[v];
  }
  __syncthreads();

  const int64_t x = x0 + cx;
  const int y = y0 + t;
  if (t < TY - 1 && y < a.n && x < nx) {
    double* out = a.out + (int64_t)y * nx + x;
    // normal-first order back to (rho, mx, my, E): the y sweep's normal momentum is my
    out[0] = (FH[0][tid] - FH[0][tid + TX]) * a.half_inv_h;
    out[2 * a.plane] = (FH[1][tid] - FH[1][tid + TX]) * a.half_inv_h;
    out[a.plane] = (FH[2][tid] - FH[2][tid + TX]) * a.half_inv_h;
    out[3 * a.plane] = (FH[3][tid] - FH[3][tid + TX]) * a.half_inv_h;
  }
}

// |u - c|, |u|, |u + c|, |v - c|, |v|, |v + c| of a 2D Euler state (c as in wave_speeds_2d).
__device__ __forceinline__ void char2_speeds(double rho, double mx, double my, double E,
                                             double gamma, double (&s)[6]) {
#pragma clang fp contract(off)
  const double r = rcp_nr(rho);
  const double u = mx * r, v = my * r;
  const double p = (gamma - 1.0) * ((E - (0.5 * mx) * u) - (0.5 * my) * v);
  const double c = sqrt_gs((gamma * p) * r);
  s[0] = __builtin_fabs(u - c);
  s[1] = __builtin_fabs(u);
  s[2] = __builtin_fabs(u + c);
  s[3] = __builtin_fabs(v - c);
  s[4] = __builtin_fabs(v);
  s[5] = __builtin_fabs(v + c);
}

__device__ __forceinline__ void block_max6(double (&s)[6], unsigned long long* slot) {
  __shared__ double red[6][4];
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const double m = wave_max(s[f]);
    if ((threadIdx.x & 63) == 0) red[f][threadIdx.x >> 6] = m;
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    const int f = threadIdx.x;
    atomic_max_pos(slot + f, fmax(fmax(red[f][0], red[f][1]), fmax(red[f][2], red[f][3])));
  }
}

// the six maxima over the cells of u into slot[0..5] (cleared beforehand)
__global__ __launch_bounds__(256) void char2_speed_kernel(const double* __restrict__ u,
                                                          int64_t N, double gamma,
                                                          unsigned long long* slot) {
  double m[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < N;
       k += (int64_t)gridDim.x * 256) {
    double s[6];
    char2_speeds(u[k], u[N + k], u[2 * N + k], u[3 * N + k], gamma, s);
#pragma unroll
    for (int f = 0; f < 6; ++f) m[f] = fmax(m[f], s[f]);
  }
  block_max6(m, slot);
}

// ------------------------------------------------------------------ host side
template <bool FUSE>
static int launch_char2(Char2Args a, hipStream_t s) {
  a.tiles = ((int64_t)a.n + C2_NT - 2) / (C2_NT - 1);
  const int64_t blocks = a.tiles * a.rows;
  if (blocks > 0x7fffffff) return set_error(WZN_ERR_SIZE, "grid too large (characteristic sweep)");
  hipLaunchKernelGGL((char2_kernel<C2_NT, FUSE>), dim3((unsigned)blocks), dim3(C2_NT), 0, s, a);
  return check_launch("char2_kernel");
}

static int launch_char2_col(Char2Args a, hipStream_t s) {
  a.tiles = ((int64_t)a.n + CY_TY - 2) / (CY_TY - 1);
  const int64_t blocks = a.tiles * ((a.rows + CY_TX - 1) / CY_TX);
  if (blocks > 0x7fffffff) return set_error(WZN_ERR_SIZE, "grid too large (characteristic sweep)");
  hipLaunchKernelGGL((char2_col_kernel<CY_TX, CY_TY>), dim3((unsigned)blocks), dim3(CY_TX * CY_TY),
                     0, s, a);
  return check_launch("char2_col_kernel");
}

static int launch_char2_speed(const double* u, int64_t N, double gamma,
                              unsigned long long* slot, hipStream_t s) {
  int64_t b = (N + 255) / 256;
  b = b > 4096 ? 4096 : (b < 1 ? 1 : b);
  hipLaunchKernelGGL(char2_speed_kernel, dim3((unsigned)b), dim3(256), 0, s, u, N, gamma, slot);
  return check_launch("char2_speed_kernel");
}

static Char2Args char2_base(const wzn_params* p, int64_t n, int64_t rows, double h, int bc) {
  Char2Args a{};
  a.n = (int)n;
  a.rows = rows;
  a.plane = n * rows;
  a.bc = bc;
  a.half_inv_h = 0.5 / h;
  a.gamma = p->gamma;
  a.eps_s = 16.0 * p->eps;
  a.Aq = 0.25 * p->A;
  return a;
}

// Where each sweep takes its alphas: from the six slots (x: 0..2, y: 3..5), a device array of
// eight, or the constants of the params.
struct Char2Alpha {
  const unsigned long long* slot6;
  const double* arr8;
};
static void set_alpha(Char2Args& a, const wzn_params* p, const Char2Alpha& al, int dir) {
  if (al.arr8) a.alpha_arr = al.arr8 + 4 * dir;
  else if (al.slot6) a.alpha_slot = al.slot6 + 3 * dir;
  else a.alpha_const = dir == 0 ? p->lf_alpha_x : p->lf_alpha_y;
}

// The y part of L(U) into work[0 .. 4 nx ny), by the column kernel.  Its workgroup 0 clears
// the six words zero6 (if given).
static int char2_ypart(const wzn_params* p, const double* u, double* work, int64_t nx,
                       int64_t ny, double dy, const Char2Alpha& al, unsigned long long* zero6,
                       hipStream_t s) {
  Char2Args ay = char2_base(p, ny, nx, dy, p->bc_y);
  ay.uin = u;
  ay.out = work;
  set_alpha(ay, p, al, 1);
  if (zero6) {
    ay.slot_zero = zero6;
    ay.zero_count = 6;
  }
  return launch_char2_col(ay, s);
}

int rhs_2d_char(const wzn_params* p, const double* u, double* dudt, double* work, int64_t nx,
                int64_t ny, double dx, double dy, const double* alpha8, Workspace* ws,
                hipStream_t s) {
  Char2Alpha al{nullptr, alpha8};
  unsigned long long* slot = ws->scratch + 64;
  if (!alpha8 && (p->lf_alpha_x < 0.0 || p->lf_alpha_y < 0.0)) {
    if (p->lf_alpha_x >= 0.0 || p->lf_alpha_y >= 0.0)
      return set_error(WZN_ERR_UNSUPPORTED, "characteristic fields: freeze both alphas or none");
    int st = launch_zero_words(slot, 6, s);
    if (st) return st;
    st = launch_char2_speed(u, nx * ny, p->gamma, slot, s);
    if (st) return st;
    al.slot6 = slot;
  }
  int st = char2_ypart(p, u, work, nx, ny, dy, al, nullptr, s);
  if (st) return st;
  Char2Args ax = char2_base(p, nx, ny, dx, p->bc_x);
  ax.uin = u;
  ax.out = dudt;
  ax.ly = work;
  ax.mode = MODE_RHS;
  set_alpha(ax, p, al, 0);
  return launch_char2<true>(ax, s);
}

// Slot protocol: a ring of three sets of six words; stage s reads the maxima of its input
// from set s % 3 (its alphas, and at the first stage of a step the dt speeds), the y sweep
// clears set (s + 2) % 3, and the x sweep maxes those of its output into set (s + 1) % 3.
int rk3_run_2d_char(const wzn_params* p, double* u, double* stage, double* work, int64_t nx,
                    int64_t ny, double dx, double dy, double cfl, int32_t nsteps,
                    const double* dt_in, double* dt_out, Workspace* ws, hipStream_t s) {
  static const double RA[3] = {0.0, 3.0 / 4.0, 1.0 / 3.0};
  static const double RB[3] = {1.0, 1.0 / 4.0, 2.0 / 3.0};
  const int64_t N = nx * ny, M = 4 * N;
  double* U1 = stage;
  double* U2 = stage + M;
  if (p->lf_alpha_x >= 0.0 || p->lf_alpha_y >= 0.0)
    return set_error(WZN_ERR_UNSUPPORTED, "characteristic runs reduce their alphas");
  unsigned long long* ring = ws->scratch + 64;
  int st = WZN_OK;
  if (nsteps > 0) {
    st = launch_zero_words(ring, 18, s);
    if (st) return st;
    st = launch_char2_speed(u, N, p->gamma, ring, s);
    if (st) return st;
  }
  int64_t sidx = 0;
  for (int32_t step = 0; step < nsteps; ++step) {
    for (int k = 0; k < 3; ++k, ++sidx) {
      const double* uin = k == 0 ? u : (k == 1 ? U1 : U2);
      double* out = k == 0 ? U1 : (k == 1 ? U2 : u);
      unsigned long long* cur = ring + 6 * (sidx % 3);
      Char2Alpha al{cur, nullptr};
      st = char2_ypart(p, uin, work, nx, ny, dy, al, ring + 6 * ((sidx + 2) % 3), s);
      if (st) return st;
      Char2Args ax = char2_base(p, nx, ny, dx, p->bc_x);
      ax.uin = uin;
      ax.out = out;
      ax.ly = work;
      ax.un = k == 0 ? nullptr : u;
      ax.mode = MODE_STAGE;
      ax.rk_a = RA[k];
      ax.rk_b = RB[k];
      set_alpha(ax, p, al, 0);
      if (dt_in) {
        ax.dt_arr = dt_in + step;
      } else if (k == 0) {
        ax.dt_speed_slot = cur;
        ax.cfl = cfl;
        ax.dx = dx;
        ax.dy = dy;
        ax.dt_slot_write = ws->dt;
      } else {
        ax.dt_slot_read = ws->dt;
      }
      if (dt_out && k == 0) ax.dt_rec = dt_out + step;
      ax.speed_next = ring + 6 * ((sidx + 1) % 3);
      st = launch_char2<true>(ax, s);
      if (st) return st;
    }
  }
  return WZN_OK;
}

}  // namespace wzn
